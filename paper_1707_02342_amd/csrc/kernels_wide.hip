// Rollout schedule "wide": a whole wavefront (64 lanes) per sample, eight samples per
// 512-thread block.  Each step carries half as many layer-2 products per lane as the
// 32-lane layout, and at K = 1920 there are two waves per SIMD.  Measured on MI355X
// it is nevertheless slower than the 32-lane layout (67.9 vs 53.2 us per iteration at
// K = 1920, T = 100): the DPP operand instructions that carry the products do not
// issue concurrently from two waves, so per sample the 64-lane layout spends more
// SIMD cycles on them.  It is kept as an explicit schedule.
//
// Lane l = 16 r + c (row r = 0..3, column c = 0..15).  Phases as in the 32-lane
// layout (noise, serial chain of the dynamic states, kinematics and cost parallel
// over t, the block's softmin partial); the chain per step:
//   layer 1: row r evaluates hidden neurons 16 s(r) + c with s = (0, 1, 1, 0)[r]; the
//            four state components sit in the lanes of each quad (component = l & 3)
//            and reach every lane through quad_perm DPP operands;
//   layer 2: row r accumulates output 16 o(r) + c with o = (0, 1, 0, 1)[r] over the 16
//            inputs of its own row (row_ror DPP operands), so rows 0 and 2 hold the two
//            halves of outputs 0..15 and rows 1 and 3 those of 16..31; one
//            v_permlane32_swap adds the halves;
//   layer 3: the lower half-wave forms outputs 0 and 1, the upper 2 and 3 (two products
//            per lane and a reduce-scatter over the half-wave); a second
//            v_permlane32_swap brings each lane its component l & 3;
//   update:  x_d += dt f in compensated (two-sum) form, one component per lane.
// The network arithmetic is the FP32 network of the other schedules with another
// summation order.
#include "wave_common.hip.h"

namespace mppi {

constexpr int kWideBlock = 512;
constexpr int kWideSlots = 8;   // samples (waves) per block

// (new first operand, new second operand) of v_permlane32_swap: the first holds the
// lower half-wave of both operands, the second the upper half.
__device__ __forceinline__ void swap_halves(float& a, float& b) {
  auto r = __builtin_amdgcn_permlane32_swap(as_u(a), as_u(b), false, false);
  a = as_f(r[0]);
  b = as_f(r[1]);
}

// Compensated exclusive scan of (hi, lo) pairs over the 64 lanes.
__device__ __forceinline__ void scan64_excl2(float& hi, float& lo, int l) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const float oh = __shfl_up(hi, d, 64);
    const float ol = __shfl_up(lo, d, 64);
    if (l >= d) {
      float s_, e_;
      two_sum(hi, oh, s_, e_);
      hi = s_;
      lo = lo + (ol + e_);
    }
  }
  const float ph = __shfl_up(hi, 1, 64);
  const float pl = __shfl_up(lo, 1, 64);
  hi = l == 0 ? 0.0f : ph;
  lo = l == 0 ? 0.0f : pl;
}

// Compensated sum of (hi, lo) over the 64 lanes, the same bits in every lane.
__device__ __forceinline__ void sum64_2(float& hi, float& lo) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const float oh = __shfl_xor(hi, m, 64);
    const float ol = __shfl_xor(lo, m, 64);
    float s_, e_;
    two_sum(hi, oh, s_, e_);
    hi = s_;
    lo = (lo + ol) + e_;
  }
}

template <int NQ>
__global__ __launch_bounds__(kWideBlock) void rollout_wide_kernel(RolloutArgs a) {
  if (a.iter_dev) a.nk.iter = *a.iter_dev;   // the device counter, advanced by the final merge
  constexpr int HID = 32;
  extern __shared__ float smem[];
  const int T = a.T;
  const int T4 = (T + 4) & ~3;
  const int eStride = (2 * T + 3) & ~3;
  float* sU = smem;                                  // [2T]
  float* sE = sU + eStride;                          // [8][2T]
  float* sX = sE + kWideSlots * eStride;             // [8][T4][4]
  float* red = sX + kWideSlots * T4 * 4;             // [8][2T]
  float* scratch = red + kWideSlots * eStride;       // [32]

  const int l = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int r = l >> 4;
  const int c = l & 15;
  const int comp = l & 3;
  const int h = l >> 5;
  const int k = blockIdx.x * kWideSlots + wv;
  const bool valid = k < a.K;
  const bool zm = k >= a.K_imp;   // exploration sample: v = eps, delta = eps - u
  float* myE = sE + wv * eStride;
  float4* myX = reinterpret_cast<float4*>(sX + wv * T4 * 4);

  for (int i = threadIdx.x; i < 2 * T; i += kWideBlock) sU[i] = a.U[i];

  // ---- per-lane network constants --------------------------------------------------
  const float* W1 = a.params;
  const float* b1 = W1 + HID * 6;
  const float* W2 = b1 + HID;
  const float* b2 = W2 + HID * HID;
  const float* W3 = b2 + HID;
  const float* b3 = W3 + 4 * HID;
  const int sIn = (r == 1 || r == 2) ? 1 : 0;        // input half of this row
  const int oOut = r & 1;                             // output half of this row
  const int jIn = 16 * sIn + c;                       // layer-1 neuron of this lane
  const int jOut = 16 * oOut + c;                     // layer-2 neuron of this lane
  float w1[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) w1[i] = W1[jIn * 6 + i];
  const float bb1 = b1[jIn];
  float w2[16];
  int src[16];
  src[0] = c;
  src[1] = ror_src<1>(c);   src[2] = ror_src<2>(c);   src[3] = ror_src<3>(c);
  src[4] = ror_src<4>(c);   src[5] = ror_src<5>(c);   src[6] = ror_src<6>(c);
  src[7] = ror_src<7>(c);   src[8] = ror_src<8>(c);   src[9] = ror_src<9>(c);
  src[10] = ror_src<10>(c); src[11] = ror_src<11>(c); src[12] = ror_src<12>(c);
  src[13] = ror_src<13>(c); src[14] = ror_src<14>(c); src[15] = ror_src<15>(c);
#pragma unroll
  for (int s = 0; s < 16; ++s) w2[s] = W2[jOut * HID + 16 * sIn + src[s]];
  const float bb2 = (h == 0) ? b2[jOut] : 0.0f;       // the bias enters one half once
  const float w3a = W3[(2 * h) * HID + jOut];
  const float w3b = W3[(2 * h + 1) * HID + jOut];
  const float b3c = b3[comp];
  const bool bit0 = (l & 1) != 0;
  const bool mine = ((l >> 1) & 1) == h;              // component l & 3 formed in this half

  float x0v[kStateDim];
#pragma unroll
  for (int i = 0; i < kStateDim; ++i) x0v[i] = a.x0_dev ? a.x0_dev[i] : a.x0[i];

  // ---- A: noise (lane l draws steps l + 64 i) ---------------------------------------
  float ea[NQ], eb[NQ];
  const int NT = (T + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    ea[i] = 0.0f;
    eb[i] = 0.0f;
    if (i < NT) {
      const int t = min(64 * i + l, T - 1);
      draw_eps((uint32_t)t, (uint32_t)k, a.nk, ea[i], eb[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int t = 64 * i + l;
    if (i < NT && t < T) {
      myE[2 * t] = ea[i];
      myE[2 * t + 1] = eb[i];
    }
  }
  Acc xd{x0v[3 + comp], 0.0f};
  if (l < 4) sX[wv * T4 * 4 + l] = x0v[3 + l];
  __syncthreads();

  // ---- B: serial chain of the dynamic states ---------------------------------------
  {
    float2 u = *reinterpret_cast<const float2*>(sU);
    float2 e = *reinterpret_cast<const float2*>(myE);
    for (int t = 0; t < T; ++t) {
      const int tn = min(t + 1, T - 1);
      const float2 u_next = *reinterpret_cast<const float2*>(sU + 2 * tn);
      const float2 e_next = *reinterpret_cast<const float2*>(myE + 2 * tn);
      const float vc0 = fminf(fmaxf(zm ? e.x : u.x + e.x, a.u_lo0), a.u_hi0);
      const float vc1 = fminf(fmaxf(zm ? e.y : u.y + e.y, a.u_lo1), a.u_hi1);
      // layer 1
      float acc1 = __builtin_fmaf(w1[4], vc0, bb1);
      acc1 = __builtin_fmaf(w1[5], vc1, acc1);
      const float xh = xd.hi;
      FMAC_DPP_FIRST(acc1, xh, w1[0], "quad_perm:[0,0,0,0]");
      FMAC_DPP(acc1, xh, w1[1], "quad_perm:[1,1,1,1]");
      FMAC_DPP(acc1, xh, w1[2], "quad_perm:[2,2,2,2]");
      FMAC_DPP(acc1, xh, w1[3], "quad_perm:[3,3,3,3]");
      const float h1 = tanh_f(acc1);
      // layer 2: half of each output's inputs, two interleaved chains
      float P = __builtin_fmaf(w2[0], h1, bb2);
      float P2 = w2[1] * dpp_f<kRowRor + 1>(h1);
      FMAC_DPP_FIRST(P, h1, w2[2], "row_ror:2");
      FMAC_DPP(P2, h1, w2[3], "row_ror:3");
      FMAC_DPP(P, h1, w2[4], "row_ror:4");
      FMAC_DPP(P2, h1, w2[5], "row_ror:5");
      FMAC_DPP(P, h1, w2[6], "row_ror:6");
      FMAC_DPP(P2, h1, w2[7], "row_ror:7");
      FMAC_DPP(P, h1, w2[8], "row_ror:8");
      FMAC_DPP(P2, h1, w2[9], "row_ror:9");
      FMAC_DPP(P, h1, w2[10], "row_ror:10");
      FMAC_DPP(P2, h1, w2[11], "row_ror:11");
      FMAC_DPP(P, h1, w2[12], "row_ror:12");
      FMAC_DPP(P2, h1, w2[13], "row_ror:13");
      FMAC_DPP(P, h1, w2[14], "row_ror:14");
      FMAC_DPP(P2, h1, w2[15], "row_ror:15");
      float lo = P + P2, hi = lo;
      swap_halves(lo, hi);
      const float h2 = tanh_f(lo + hi);
      // layer 3: outputs 2h and 2h + 1 over the half-wave, reduce-scattered
      const float pa = w3a * h2, pb = w3b * h2;
      const float send = bit0 ? pa : pb, keep = bit0 ? pb : pa;
      float g = keep + dpp_f<kQuadXor1>(send);                 // output 2h + bit0
      g = g + dpp_f<kQuadXor2>(g);
      g = g + dpp_f<kRowRor + 8>(g);
      g = g + dpp_f<kRowRor + 4>(g);
      g = add_rows(g);
      float glo = g, ghi = g;
      swap_halves(glo, ghi);                                   // lower / upper half's value
      const float f = (mine ? g : (h ? glo : ghi)) + b3c;
      xd.add(a.dt * f);
      if (l < 4) sX[wv * T4 * 4 + (t + 1) * 4 + l] = xd.value();
      u = u_next;
      e = e_next;
    }
  }
  __syncthreads();

  // ---- C: kinematics and cost, parallel over t (lane l owns steps [l npl, (l+1) npl)) --
  const int npl = NT;
  const int tb = l * npl;
  float th_h = 0.0f, th_l = 0.0f;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = tb + q;
    if (q < npl && t < T) {
      float s_, e_;
      two_sum(th_h, a.dt * myX[t].w, s_, e_);
      th_h = s_;
      th_l += e_;
    }
  }
  scan64_excl2(th_h, th_l, l);
  {
    float s_, e_;
    two_sum(x0v[2], th_h, s_, e_);
    th_h = s_;
    th_l = th_l + e_;
  }
  float dpx[NQ], dpy[NQ];
  float px_h = 0.0f, px_l = 0.0f, py_h = 0.0f, py_l = 0.0f;
  {
    float th = th_h, thl = th_l;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      dpx[q] = 0.0f;
      dpy[q] = 0.0f;
      const int t = tb + q;
      if (q < npl && t < T) {
        const float4 xs = myX[t];
        float sn, cs;
        sincosf(th + thl, &sn, &cs);
        dpx[q] = a.dt * (cs * xs.y - sn * xs.z);
        dpy[q] = a.dt * (sn * xs.y + cs * xs.z);
        float s_, e_;
        two_sum(px_h, dpx[q], s_, e_);
        px_h = s_;
        px_l += e_;
        two_sum(py_h, dpy[q], s_, e_);
        py_h = s_;
        py_l += e_;
        two_sum(th, a.dt * xs.w, s_, e_);
        th = s_;
        thl += e_;
      }
    }
  }
  scan64_excl2(px_h, px_l, l);
  scan64_excl2(py_h, py_l, l);
  {
    float s_, e_;
    two_sum(x0v[0], px_h, s_, e_);
    px_h = s_;
    px_l += e_;
    two_sum(x0v[1], py_h, s_, e_);
    py_h = s_;
    py_l += e_;
  }
  float pxh[NQ], pxl[NQ], pyh[NQ], pyl[NQ], th1[NQ];
  {
    float th = th_h, thl = th_l;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int t = tb + q;
      if (q < npl && t < T) {
        float s_, e_;
        two_sum(px_h, dpx[q], s_, e_);
        px_h = s_;
        px_l += e_;
        two_sum(py_h, dpy[q], s_, e_);
        py_h = s_;
        py_l += e_;
        two_sum(th, a.dt * myX[t].w, s_, e_);
        th = s_;
        thl += e_;
      }
      pxh[q] = px_h;
      pxl[q] = px_l;
      pyh[q] = py_h;
      pyl[q] = py_l;
      th1[q] = th + thl;
    }
  }
  float mv[NQ][4], fxv[NQ], fyv[NQ], dec[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    int idx[4];
    map_taps(a.cost, pxh[q], pxl[q], pyh[q], pyl[q], idx, fxv[q], fyv[q]);
#pragma unroll
    for (int i = 0; i < 4; ++i) mv[q][i] = a.map[idx[i]];
    dec[q] = a.decay[min(tb + q, T - 1) + 1];
  }
  Acc Sacc{0.0f, 0.0f};
  bool ok = true;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = tb + q;
    if (q < npl && t < T) {
      const float4 xn = myX[t + 1];
      const float px1 = pxh[q] + pxl[q], py1 = pyh[q] + pyl[q];
      Sacc.add(state_cost_h(a.cost, bilerp(mv[q], fxv[q], fyv[q]), dec[q], xn.y, xn.z));
      const float u0 = sU[2 * t], u1 = sU[2 * t + 1];
      const float d0 = zm ? myE[2 * t] - u0 : myE[2 * t];
      const float d1 = zm ? myE[2 * t + 1] - u1 : myE[2 * t + 1];
      Sacc.add(a.gcs0 * (u0 * d0) + a.gcs1 * (u1 * d1));
      ok = ok && finite_f(px1) && finite_f(py1) && finite_f(th1[q]) && finite_f(xn.x) &&
           finite_f(xn.y) && finite_f(xn.z) && finite_f(xn.w);
    }
  }
  float S_h = Sacc.hi, S_l = Sacc.lo;
  sum64_2(S_h, S_l);
  float S = S_h + S_l;
  int okc = ok ? 1 : 0;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) okc &= __shfl_xor(okc, m, 64);
  if (!valid || !okc || !finite_f(S)) S = kInf;
  if (valid && l == 0) store_through(a.S + k, S);   // read by the host or Algorithm 3's update

  if (a.cem_zeta > 0) {
    // Algorithm 3: the sample's delta row, for the elite average
    if (valid) {
      float* drow = a.D + (size_t)k * 2 * T;
      for (int o = l; o < 2 * T; o += 64) drow[o] = zm ? myE[o] - sU[o] : myE[o];
    }
    return;   // the cross-entropy update runs in the launch that follows
  }

  // ---- D: softmin partial of the block's samples ------------------------------------
  if (l == 0) scratch[wv] = S;
  __syncthreads();
  float rho = scratch[0];
#pragma unroll
  for (int i = 1; i < kWideSlots; ++i) rho = fminf(rho, scratch[i]);
  const float e = rel_weight(S, rho, a.inv_lambda);
  if (l == 0) scratch[kWideSlots + wv] = e;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int t = 64 * i + l;
    if (i < NT && t < T) {
      const float d0 = zm ? ea[i] - sU[2 * t] : ea[i];
      const float d1 = zm ? eb[i] - sU[2 * t + 1] : eb[i];
      red[wv * eStride + 2 * t] = e * d0;
      red[wv * eStride + 2 * t + 1] = e * d1;
    }
  }
  __syncthreads();
  float* N_lds = sE;   // the noise rows are no longer read
  for (int o = threadIdx.x; o < 2 * T; o += kWideBlock) {
    float s = red[o];
#pragma unroll
    for (int w = 1; w < kWideSlots; ++w) s += red[w * eStride + o];
    N_lds[o] = s;
  }
  float eta = scratch[kWideSlots];
#pragma unroll
  for (int w = 1; w < kWideSlots; ++w) eta += scratch[kWideSlots + w];
  finish_iteration<kWideBlock, kModelNet, true, 32>(a, blockIdx.x, rho, eta, N_lds, red);
}

template __global__ void rollout_wide_kernel<2>(RolloutArgs);
template __global__ void rollout_wide_kernel<4>(RolloutArgs);

// Dynamic LDS bytes the wide kernel needs for horizon T.
size_t wide_smem_bytes(int T) {
  const size_t e = (size_t)((2 * T + 3) & ~3);
  const size_t T4 = (size_t)((T + 4) & ~3);
  return sizeof(float) * (e + kWideSlots * e + kWideSlots * T4 * 4 + kWideSlots * e + 32);
}

}  // namespace mppi
