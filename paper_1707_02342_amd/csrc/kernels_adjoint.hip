// Adjoint rollout: gradient of the free-energy objective
//   J = -lambda log((1/K) sum_k exp(-S_k/lambda)) = rho - lambda log(eta~/K)
// (the Monte-Carlo estimate of -lambda times the free energy, Eq. FreeEnergy) with
// respect to the nominal controls U and every parameter of the dynamics network.
//
// dJ/dS_k = w_k (the weights of Algorithm 2), so every sample's reverse sweep is
// seeded with w_k and the per-sample gradients add up directly.  The layout is the
// forward "wave" layout: 32 lanes per sample, lane (row r, column c) owning hidden
// unit j = 16 r + c, two samples per wavefront, eight per block.
//
// Memory: the forward pass stored the full state every `ckpt_every` steps.  The
// sweep walks the segments backwards; for each it re-runs the segment forward from
// its checkpoint (network, kinematics and cost gradient, keeping each step's hidden
// activations in registers and the per-step scalars in LDS) and then applies the
// reverse-mode recurrences step by step:
//   p <- p + w_k grad c(x_{t+1});  a3 = dt p[3:7];  dW3 += a3 h2^T;  a2 = (W3^T a3)(1-h2^2);
//   dW2 += a2 h1^T;  a1 = (W2^T a2)(1-h1^2);  dW1 += a1 in^T;  g_in = W1^T a1;
//   dJ/du_t += g'(v_t) g_in[4:6];  p <- (dF/dx_t)^T p.
// The control-cost term gamma eps_t / Sigma weighted by w_k sums to gamma Delta_t / Sigma
// and is added by the final reduction.  Layer 2's two products (dW2 and W2^T a2) read
// the other lanes' a2 through row_ror DPP operands, as the forward pass does.
#include "wave_common.hip.h"

namespace mppi {

constexpr int kAdjMaxSeg = 16;
constexpr int kSegStride = 20;   // per-step scalars: x(7) v(2) vc(2) cos sin gc(7)
constexpr int kNP32 = 1412;      // parameters of the 6-32-32-4 network

// Sum of v over the sample's 32 lanes, the same bits in every lane.
__device__ __forceinline__ float allsum32(float v) {
  v = v + dpp_f<kRowRor + 8>(v);
  v = v + dpp_f<kRowRor + 4>(v);
  v = v + dpp_f<kRowRor + 2>(v);
  v = v + dpp_f<kRowRor + 1>(v);
  return add_rows(v);
}

size_t adjoint_smem_bytes(int T, int ckpt_every) {
  return sizeof(float) * (2 * (size_t)T + kWaveSlots * (size_t)ckpt_every * kSegStride +
                          kWaveSlots * 2 * (size_t)kAdjMaxSeg + kWaveSlots * 2 * (size_t)T + 4 * kNP32 + 16);
}

__global__ __launch_bounds__(kWaveBlock) void adjoint_wave_kernel(AdjointArgs a) {
  constexpr int HID = 32;
  extern __shared__ float smem[];
  const int T = a.T, C = a.ckpt_every;
  float* sU = smem;                                    // [2T]
  float* sSeg = sU + 2 * T;                            // [8][C][20]
  float* sEps = sSeg + kWaveSlots * C * kSegStride;    // [8][kAdjMaxSeg][2]
  float* sGU = sEps + kWaveSlots * 2 * kAdjMaxSeg;     // [8][T][2]
  float* sRed = sGU + kWaveSlots * 2 * T;              // [4][1412]
  float* scratch = sRed + 4 * kNP32;                   // [16]

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int half = lane >> 5;
  const int c32 = lane & 31;
  const int r = c32 >> 4;
  const int col = lane & 15;
  const int slot = wv * 2 + half;
  const int k = blockIdx.x * kWaveSlots + slot;
  const bool valid = k < a.K;
  float* mySeg = sSeg + slot * C * kSegStride;
  float* myEps = sEps + slot * 2 * kAdjMaxSeg;
  float* myGU = sGU + slot * 2 * T;

  for (int i = threadIdx.x; i < 2 * T; i += kWaveBlock) sU[i] = a.U[i];
  for (int i = c32; i < 2 * T; i += 32) myGU[i] = 0.0f;

  // ---- network constants of this lane ----------------------------------------------
  const float* W1 = a.params;
  const float* b1 = W1 + HID * 6;
  const float* W2 = b1 + HID;
  const float* b2 = W2 + HID * HID;
  const float* W3 = b2 + HID;
  const float* b3 = W3 + 4 * HID;
  const int j = 16 * r + col;
  float w1[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) w1[i] = W1[j * 6 + i];
  const float bb1 = b1[j];
  int src[16];
  src[0] = col;
  src[1] = ror_src<1>(col);   src[2] = ror_src<2>(col);   src[3] = ror_src<3>(col);
  src[4] = ror_src<4>(col);   src[5] = ror_src<5>(col);   src[6] = ror_src<6>(col);
  src[7] = ror_src<7>(col);   src[8] = ror_src<8>(col);   src[9] = ror_src<9>(col);
  src[10] = ror_src<10>(col); src[11] = ror_src<11>(col); src[12] = ror_src<12>(col);
  src[13] = ror_src<13>(col); src[14] = ror_src<14>(col); src[15] = ror_src<15>(col);
  float wP[16], wQ[16], wBo[16], wBx[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    wP[s] = W2[col * HID + 16 * r + src[s]];
    wQ[s] = W2[(16 + col) * HID + 16 * r + src[s]];
    wBo[s] = W2[(16 * r + src[s]) * HID + j];          // W2[i][j], i in this row
    wBx[s] = W2[(16 * (1 - r) + src[s]) * HID + j];    // W2[i][j], i in the other row
  }
  const float bP = (r == 0) ? b2[col] : 0.0f;
  const float bQ = (r == 1) ? b2[16 + col] : 0.0f;
  float w3[4], bb3[4];
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    w3[o] = W3[o * HID + j];
    bb3[o] = b3[o];
  }

  // ---- weight of this sample ---------------------------------------------------------
  const float rho = a.stats[0], eta = a.stats[1];
  const float Sk = valid ? a.S[k] : kInf;
  const float wk = (Sk < kInf && rho < kInf && eta > 0.0f) ? expf(-(Sk - rho) * a.inv_lambda) / eta : 0.0f;

  // ---- accumulators -----------------------------------------------------------------
  float gW1[6] = {0, 0, 0, 0, 0, 0}, gb1 = 0.0f, gb2 = 0.0f;
  float gW2o[16], gW2x[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    gW2o[s] = 0.0f;
    gW2x[s] = 0.0f;
  }
  float gW3[4] = {0, 0, 0, 0}, gb3[4] = {0, 0, 0, 0};
  float pa[kStateDim] = {0, 0, 0, 0, 0, 0, 0};
  __syncthreads();

  const int nseg = (T + C - 1) / C;
  const int n_ckpt = a.n_ckpt;
  for (int sgi = nseg - 1; sgi >= 0; --sgi) {
    const int t0 = sgi * C;
    const int n = min(C, T - t0);
    // noise of the segment, one step per lane
    if (c32 < n) {
      float e0, e1;
      draw_eps((uint32_t)(t0 + c32), (uint32_t)k, a.nk, e0, e1);
      myEps[2 * c32] = e0;
      myEps[2 * c32 + 1] = e1;
    }
    __syncthreads();
    // ---- forward re-run of the segment from its checkpoint ----
    float x[kStateDim];
    const float* cp = a.ckpt + ((size_t)(valid ? k : 0) * n_ckpt + sgi) * kCkptStride;
    // a sample with zero weight contributes nothing; it re-runs from the zero state so
    // that no non-finite value of its own trajectory can reach the sums
    const bool live = wk > 0.0f;
#pragma unroll
    for (int i = 0; i < kStateDim; ++i) x[i] = live ? cp[i] : 0.0f;
    float h1s[kAdjMaxSeg], h2s[kAdjMaxSeg];
#pragma unroll
    for (int q = 0; q < kAdjMaxSeg; ++q) {
      h1s[q] = 0.0f;
      h2s[q] = 0.0f;
      if (q < n) {
        const int t = t0 + q;
        const float u0 = sU[2 * t], u1 = sU[2 * t + 1];
        const float v0 = u0 + myEps[2 * q], v1 = u1 + myEps[2 * q + 1];
        const float vc0 = fminf(fmaxf(v0, a.u_lo0), a.u_hi0);
        const float vc1 = fminf(fmaxf(v1, a.u_lo1), a.u_hi1);
        float acc = bb1;
        acc = __builtin_fmaf(w1[0], x[3], acc);
        acc = __builtin_fmaf(w1[1], x[4], acc);
        acc = __builtin_fmaf(w1[2], x[5], acc);
        acc = __builtin_fmaf(w1[3], x[6], acc);
        acc = __builtin_fmaf(w1[4], vc0, acc);
        acc = __builtin_fmaf(w1[5], vc1, acc);
        const float h1 = tanh_f(acc);
        float P = __builtin_fmaf(wP[0], h1, bP);
        float Q = __builtin_fmaf(wQ[0], h1, bQ);
        float P2 = wP[1] * dpp_f<kRowRor + 1>(h1);
        float Q2 = wQ[1] * dpp_f<kRowRor + 1>(h1);
        FMAC_DPP_FIRST(P, h1, wP[2], "row_ror:2");
        FMAC_DPP(Q, h1, wQ[2], "row_ror:2");
        FMAC_DPP(P2, h1, wP[3], "row_ror:3");
        FMAC_DPP(Q2, h1, wQ[3], "row_ror:3");
        FMAC_DPP(P, h1, wP[4], "row_ror:4");
        FMAC_DPP(Q, h1, wQ[4], "row_ror:4");
        FMAC_DPP(P2, h1, wP[5], "row_ror:5");
        FMAC_DPP(Q2, h1, wQ[5], "row_ror:5");
        FMAC_DPP(P, h1, wP[6], "row_ror:6");
        FMAC_DPP(Q, h1, wQ[6], "row_ror:6");
        FMAC_DPP(P2, h1, wP[7], "row_ror:7");
        FMAC_DPP(Q2, h1, wQ[7], "row_ror:7");
        FMAC_DPP(P, h1, wP[8], "row_ror:8");
        FMAC_DPP(Q, h1, wQ[8], "row_ror:8");
        FMAC_DPP(P2, h1, wP[9], "row_ror:9");
        FMAC_DPP(Q2, h1, wQ[9], "row_ror:9");
        FMAC_DPP(P, h1, wP[10], "row_ror:10");
        FMAC_DPP(Q, h1, wQ[10], "row_ror:10");
        FMAC_DPP(P2, h1, wP[11], "row_ror:11");
        FMAC_DPP(Q2, h1, wQ[11], "row_ror:11");
        FMAC_DPP(P, h1, wP[12], "row_ror:12");
        FMAC_DPP(Q, h1, wQ[12], "row_ror:12");
        FMAC_DPP(P2, h1, wP[13], "row_ror:13");
        FMAC_DPP(Q2, h1, wQ[13], "row_ror:13");
        FMAC_DPP(P, h1, wP[14], "row_ror:14");
        FMAC_DPP(Q, h1, wQ[14], "row_ror:14");
        FMAC_DPP(P2, h1, wP[15], "row_ror:15");
        FMAC_DPP(Q2, h1, wQ[15], "row_ror:15");
        P = P + P2;
        Q = Q + Q2;
        swap_rows(P, Q);
        const float h2 = tanh_f(P + Q);
        float f[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) f[o] = allsum32(w3[o] * h2) + bb3[o];
        float sth, cth;
        sincosf(x[2], &sth, &cth);
        float xn[kStateDim];
        xn[0] = x[0] + a.dt * (cth * x[4] - sth * x[5]);
        xn[1] = x[1] + a.dt * (sth * x[4] + cth * x[5]);
        xn[2] = x[2] + a.dt * x[6];
#pragma unroll
        for (int i = 0; i < 4; ++i) xn[3 + i] = x[3 + i] + a.dt * f[i];
        float gpx, gpy, gvx, gvy;
        state_cost_grad(a.cost, a.map, xn[0], xn[1], xn[4], xn[5], gpx, gpy, gvx, gvy);
        if (c32 == 0) {
          float* row = mySeg + q * kSegStride;
#pragma unroll
          for (int i = 0; i < kStateDim; ++i) row[i] = x[i];
          row[7] = v0;
          row[8] = v1;
          row[9] = vc0;
          row[10] = vc1;
          row[11] = cth;
          row[12] = sth;
          row[13] = wk * gpx;
          row[14] = wk * gpy;
          row[15] = 0.0f;
          row[16] = 0.0f;
          row[17] = wk * gvx;
          row[18] = wk * gvy;
          row[19] = 0.0f;
        }
        h1s[q] = h1;
        h2s[q] = h2;
#pragma unroll
        for (int i = 0; i < kStateDim; ++i) x[i] = xn[i];
      }
    }
    __syncthreads();
    // ---- reverse sweep of the segment ----
#pragma unroll
    for (int q = kAdjMaxSeg - 1; q >= 0; --q) {
      if (q < n) {
        const int t = t0 + q;
        const float* row = mySeg + q * kSegStride;
        pa[0] += row[13];
        pa[1] += row[14];
        pa[4] += row[17];
        pa[5] += row[18];
        const float h1 = h1s[q], h2 = h2s[q];
        float a3[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
          a3[o] = a.dt * pa[3 + o];
          gb3[o] += a3[o];
          gW3[o] = __builtin_fmaf(a3[o], h2, gW3[o]);
        }
        float gh2 = w3[0] * a3[0];
        gh2 = __builtin_fmaf(w3[1], a3[1], gh2);
        gh2 = __builtin_fmaf(w3[2], a3[2], gh2);
        gh2 = __builtin_fmaf(w3[3], a3[3], gh2);
        const float a2 = gh2 * (1.0f - h2 * h2);
        gb2 += a2;
        float xa = a2, ya = a2;
        swap_rows(xa, ya);
        const float a2x = (r == 0) ? ya : xa;            // a2 of the other row, same column
        gW2o[0] = __builtin_fmaf(a2, h1, gW2o[0]);
        gW2x[0] = __builtin_fmaf(a2x, h1, gW2x[0]);
        float gh1a = a2 * wBo[0];
        float gh1b = a2x * wBx[0];
        FMAC_DPP_FIRST(gW2o[1], a2, h1, "row_ror:1");
        FMAC_DPP_FIRST(gW2x[1], a2x, h1, "row_ror:1");
        FMAC_DPP(gh1a, a2, wBo[1], "row_ror:1");
        FMAC_DPP(gh1b, a2x, wBx[1], "row_ror:1");
#define ADJ_STEP(S)                                        \
  FMAC_DPP(gW2o[S], a2, h1, "row_ror:" #S);                \
  FMAC_DPP(gW2x[S], a2x, h1, "row_ror:" #S);               \
  FMAC_DPP(gh1a, a2, wBo[S], "row_ror:" #S);               \
  FMAC_DPP(gh1b, a2x, wBx[S], "row_ror:" #S);
        ADJ_STEP(2) ADJ_STEP(3) ADJ_STEP(4) ADJ_STEP(5) ADJ_STEP(6) ADJ_STEP(7) ADJ_STEP(8)
        ADJ_STEP(9) ADJ_STEP(10) ADJ_STEP(11) ADJ_STEP(12) ADJ_STEP(13) ADJ_STEP(14) ADJ_STEP(15)
#undef ADJ_STEP
        const float a1 = (gh1a + gh1b) * (1.0f - h1 * h1);
        gb1 += a1;
        const float in[6] = {row[3], row[4], row[5], row[6], row[9], row[10]};
        float gin[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          gW1[i] = __builtin_fmaf(a1, in[i], gW1[i]);
          gin[i] = allsum32(w1[i] * a1);
        }
        if (c32 == 0) {
          const float v0 = row[7], v1 = row[8];
          myGU[2 * t] = (v0 > a.u_lo0 && v0 < a.u_hi0) ? gin[4] : 0.0f;
          myGU[2 * t + 1] = (v1 > a.u_lo1 && v1 < a.u_hi1) ? gin[5] : 0.0f;
        }
        // p_t = (dF/dx_t)^T p_{t+1}
        const float cth = row[11], sth = row[12], vx = row[4], vy = row[5];
        const float np2 = pa[2] + a.dt * (pa[0] * (-sth * vx - cth * vy) + pa[1] * (cth * vx - sth * vy));
        const float np3 = pa[3] + gin[0];
        const float np4 = pa[4] + a.dt * (pa[0] * cth + pa[1] * sth) + gin[1];
        const float np5 = pa[5] + a.dt * (-pa[0] * sth + pa[1] * cth) + gin[2];
        const float np6 = pa[6] + a.dt * pa[2] + gin[3];
        pa[2] = np2;
        pa[3] = np3;
        pa[4] = np4;
        pa[5] = np5;
        pa[6] = np6;
      }
    }
    __syncthreads();
  }

  // ---- block reduction of the parameter gradients -------------------------------------
  // Lane (r, c) of every sample holds the same parameter entries, so the two samples
  // of a wave are added through a cross-half shuffle and the four waves through LDS.
  auto pair = [&](float v) { return v + __shfl_xor(v, 32, 64); };
  float* red = sRed + wv * kNP32;
  // every value is paired by all 64 lanes (the shuffle needs them all), half 0 stores
  float vals[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) vals[i] = pair(gW1[i]);
  if (half == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) red[j * 6 + i] = vals[i];
  }
  const float vb1 = pair(gb1);
  if (half == 0) red[192 + j] = vb1;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const float vo = pair(gW2o[s]);
    const float vx2 = pair(gW2x[s]);
    if (half == 0) {
      red[224 + (16 * r + src[s]) * HID + j] = vo;
      red[224 + (16 * (1 - r) + src[s]) * HID + j] = vx2;
    }
  }
  const float vb2 = pair(gb2);
  if (half == 0) red[1248 + j] = vb2;
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    const float v = pair(gW3[o]);
    if (half == 0) red[1280 + o * HID + j] = v;
  }
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    const float v = pair(gb3[o]);
    if (lane == 0) red[1408 + o] = v;
  }
  __syncthreads();
  const int stride = kNP32 + 2 * T;
  float* out = a.gpart + (size_t)blockIdx.x * stride;
  for (int i = threadIdx.x; i < kNP32; i += kWaveBlock)
    out[i] = ((sRed[i] + sRed[kNP32 + i]) + sRed[2 * kNP32 + i]) + sRed[3 * kNP32 + i];
  for (int o = threadIdx.x; o < 2 * T; o += kWaveBlock) {
    float acc = 0.0f;
#pragma unroll
    for (int sl = 0; sl < kWaveSlots; ++sl) acc += sGU[sl * 2 * T + o];
    out[kNP32 + o] = acc;
  }
}

// Sum of the G per-block gradient partials [G][stride] in two passes with a fixed
// order.  Pass 1: row chunk y (rows [y G / R, (y+1) G / R)) of 64 columns per block;
// the four waves take every fourth row of the chunk and their sums are added in wave
// order.  Pass 2: the R chunk sums in chunk order, plus the control-cost term
// gamma * Delta_t / Sigma_ii of dJ/du_t.
__global__ __launch_bounds__(256) void adjoint_reduce_partial_kernel(const float* __restrict__ gpart, int G,
                                                                     int stride, int R,
                                                                     float* __restrict__ partial) {
  __shared__ float red[4][64];
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int sub = threadIdx.x >> 6;
  const int y = blockIdx.y;
  const int g0 = (int)(((long long)y * G) / R), g1 = (int)(((long long)(y + 1) * G) / R);
  float acc = 0.0f;
  if (col < stride)
    for (int g = g0 + sub; g < g1; g += 4) acc += __builtin_nontemporal_load(gpart + (size_t)g * stride + col);
  red[sub][threadIdx.x & 63] = acc;
  __syncthreads();
  if (sub == 0 && col < stride) {
    const int c = threadIdx.x;
    partial[(size_t)y * stride + col] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
  }
}

__global__ __launch_bounds__(256) void adjoint_reduce_final_kernel(const float* __restrict__ partial, int R,
                                                                   int T, const float* __restrict__ stats,
                                                                   float gcs0, float gcs1, float* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int stride = kNP32 + 2 * T;
  if (i >= stride) return;
  float acc = 0.0f;
  for (int y = 0; y < R; ++y) acc += partial[(size_t)y * stride + i];
  if (i >= kNP32) {
    const int o = i - kNP32;
    acc += ((o & 1) ? gcs1 : gcs0) * stats[2 + o];
  }
  out[i] = acc;
}

}  // namespace mppi
