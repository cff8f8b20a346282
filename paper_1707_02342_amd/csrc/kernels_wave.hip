// Rollout schedule "wave": 32 lanes per sample, two samples per wavefront, for the
// latency-bound regime (a few thousand samples, e.g. K = 1920, T = 100), where one
// lane per sample would leave most of the chip idle while each lane walks a
// 100-step serial chain.
//
// Only the dynamic states x_d = (roll, v_x, v_y, theta_dot) form a serial chain: the
// network reads x_d and the control, never the pose (Section VI-B).  So the kernel
// splits each sample's work into four phases:
//
//  A. noise: each of the sample's 32 lanes draws eps for steps t = lane + 32 i
//     (Philox + Box-Muller), kept in registers and copied to LDS;
//  B. the serial x_d chain, one network evaluation per step with the 32 hidden
//     units spread one per lane:
//       layer 1: lane (row r, column c) owns neuron j = 16 r + c; the four state
//                components live in the lanes of each quad (component = lane & 3) and
//                reach every lane through quad_perm DPP operands of v_fmac_f32;
//       layer 2: each lane accumulates two outputs (c and 16 + c) over the 16 inputs
//                of its own row, reading them with row_ror DPP operands of
//                v_fmac_f32; v_permlane16_swap then exchanges the half sums between
//                the sample's two rows, so lane (r, c) ends with neuron 16 r + c;
//       layer 3: four products per lane, a reduce-scatter over each row (quad_perm
//                exchanges for bits 0 and 1 of the lane, row_ror 8 and 4 for bits 3
//                and 2) leaves output (lane & 3) in every lane, and a second
//                permlane16 swap adds the two rows;
//       update:  x_d += dt f in compensated (two-sum) form, one component per lane;
//     with the basis-function model (MODEL = kModelBasis) phase A also forms, for
//     each of the lane's steps, everything that depends on the control alone (sin and
//     tan of the steering and the four basis functions of the throttle and steering
//     only, times Theta) into LDS; in the chain the four state components reach every
//     lane of the quad through quad_perm DPP moves, every lane forms the 21 raw products
//     of the state (normalisers folded into its column of Theta) and lane (component c)
//     sums its own output: no cross-lane reduction and no transcendental on the chain;
//  C. kinematics and cost, lane-parallel over t: theta and the position are prefix
//     sums of their Euler increments (scans across the 32 lanes), then the cost at
//     every post-step state and the control-cost term, summed over t;
//  D. the block's softmin partial (rho_g, eta_g, N_g) for the merge kernel.
//
// The network arithmetic of phase B is exactly the FP32 network of the lane
// schedule with a different summation order.
#include "wave_common.hip.h"

namespace mppi {

template <int HID, int NQ, int MODEL>
__global__ __launch_bounds__(kWaveBlock) void rollout_wave_kernel(RolloutArgs a) {
  if (a.iter_dev) a.nk.iter = *a.iter_dev;   // the device counter, advanced by the final merge
  static_assert(HID == 32, "the wave schedule maps 32 hidden units onto 32 lanes");
  extern __shared__ float smem[];
  // Up to 128 steps (NQ = 4) the chain stores the uncompensated state hi_t and each
  // increment y_t, and phase C forms the compensated sums from them lane-parallel;
  // beyond (NQ = 8) the chain keeps the compensation itself (less LDS per block).
  constexpr bool kDefer = NQ <= 4;
  constexpr int kXW = kDefer ? 8 : 4;                // floats per step in sX
  constexpr bool kNetV = MODEL == kModelNet;         // the chain reads the clamped controls from sV
  const int T = a.T;
  const int T4 = (T + 4) & ~3;                       // padded row counts (16-byte aligned)
  const int eStride = (2 * T + 3) & ~3;
  float* sU = smem;                                  // [2T]
  float* sE = sU + eStride;                          // [8][2T] noise
  float* sV = sE + kWaveSlots * eStride;             // network model: [8][2T] clamped controls g(v)
  float* sX = sV + (kNetV ? kWaveSlots * eStride : 0);   // [8][T4][kXW]
  // [4][2T] wave partials of phase D (in the deferred layout they reuse sX, which phase C
  // has finished reading before the barrier that precedes them)
  float* red = kDefer ? sX : sX + kWaveSlots * T4 * kXW;
  float* scratch = kDefer ? sX + kWaveSlots * T4 * kXW : red + 4 * eStride;   // [16]
  float* sB = scratch + 16;                          // basis model: [8][T][8] control terms

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int half = lane >> 5;
  const int c32 = lane & 31;
  const int r = c32 >> 4;
  const int col = lane & 15;
  const int comp = lane & 3;
  const int slot = wv * 2 + half;
  const int k = blockIdx.x * kWaveSlots + slot;
  const bool valid = k < a.K;
  const bool zm = k >= a.K_imp;   // exploration sample: v = eps, delta = eps - u
  float* myE = sE + slot * eStride;
  float* myV = sV + slot * eStride;
  float4* myX = reinterpret_cast<float4*>(sX + slot * T4 * kXW);   // [T4] (NQ = 8) or [T4][2] (hi, y)

  for (int i = threadIdx.x; i < 2 * T; i += kWaveBlock) sU[i] = a.U[i];

  // ---- per-lane network constants (network model only: with the basis-function
  // model params holds Theta, and none of these is read) --------------------------
  constexpr bool kNet = MODEL == kModelNet;
  const float* W1 = a.params;
  const float* b1 = W1 + HID * 6;
  const float* W2 = b1 + HID;
  const float* b2 = W2 + HID * HID;
  const float* W3 = b2 + HID;
  const float* b3 = W3 + 4 * HID;
  const int j = 16 * r + col;
  // layers 1 and 2 form tanh's argument already multiplied by 2 log2(e)
  float w1[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) w1[i] = kNet ? kTanhScale * W1[j * 6 + i] : 0.0f;
  const float bb1 = kNet ? kTanhScale * b1[j] : 0.0f;
  float wP[16], wQ[16];
  int src[16];
  src[0] = col;
  src[1] = ror_src<1>(col);   src[2] = ror_src<2>(col);   src[3] = ror_src<3>(col);
  src[4] = ror_src<4>(col);   src[5] = ror_src<5>(col);   src[6] = ror_src<6>(col);
  src[7] = ror_src<7>(col);   src[8] = ror_src<8>(col);   src[9] = ror_src<9>(col);
  src[10] = ror_src<10>(col); src[11] = ror_src<11>(col); src[12] = ror_src<12>(col);
  src[13] = ror_src<13>(col); src[14] = ror_src<14>(col); src[15] = ror_src<15>(col);
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    wP[s] = kNet ? kTanhScale * W2[col * HID + 16 * r + src[s]] : 0.0f;
    wQ[s] = kNet ? kTanhScale * W2[(16 + col) * HID + 16 * r + src[s]] : 0.0f;
  }
  const float bP = (kNet && r == 0) ? kTanhScale * b2[col] : 0.0f;
  const float bQ = (kNet && r == 1) ? kTanhScale * b2[16 + col] : 0.0f;
  // layer 3 times dt, as a reduce-scatter over each quad with the weights placed per lane:
  // lane L keeps output oA = L & 3 (its final one) and oB = oA ^ 2 (passed on in the second
  // exchange), and sends outputs oA ^ 1 and oA ^ 3 to its partner L ^ 1, whose oA and oB they
  // are; dt b3 enters once per output, in the lanes 0..3 of each sample
  const float wKA = kNet ? a.dt * W3[comp * HID + j] : 0.0f;
  const float wKB = kNet ? a.dt * W3[(comp ^ 2) * HID + j] : 0.0f;
  const float wSA = kNet ? a.dt * W3[(comp ^ 1) * HID + j] : 0.0f;
  const float wSB = kNet ? a.dt * W3[(comp ^ 3) * HID + j] : 0.0f;
  const float bKA = (kNet && c32 < 4) ? a.dt * b3[comp] : 0.0f;
  // basis-function model: this lane's column of Theta with each basis function's
  // normaliser folded in (the chain multiplies raw products such as sin(u_delta) tan(alpha_f))
  constexpr int kRaw = 21;
  constexpr int kRawIdx[kRaw] = {1, 2, 3, 4, 5, 6, 7, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22};
  constexpr float kRawScale[kRaw] = {0.1f, 1.0f / 1200.0f, 1.0f / (1200.0f * 1200.0f),
                                     1.0f / (1200.0f * 1200.0f * 1200.0f), 1.0f / 25.0f, 0.1f, 0.1f,
                                     1.0f / 40.0f, 1.0f / 1400.0f, 1.0f / (1400.0f * 1400.0f),
                                     1.0f / (1400.0f * 1400.0f * 1400.0f), 1.0f / 40.0f,
                                     1.0f / (40.0f * 40.0f), 1.0f / (40.0f * 40.0f * 40.0f), 1.0f / 50.0f,
                                     1.0f, 1.0f, 1.0f / 3.0f, 0.2f, 0.01f, 0.001f};
  float kc[kRaw];
#pragma unroll
  for (int i = 0; i < kRaw; ++i) kc[i] = kNet ? 0.0f : a.params[kRawIdx[i] * 4 + comp] * kRawScale[i];

  float x0v[kStateDim];
#pragma unroll
  for (int i = 0; i < kStateDim; ++i) x0v[i] = a.x0_dev ? a.x0_dev[i] : a.x0[i];

  // ---- A: noise ---------------------------------------------------------------------
  // (draws for steps past T use a clamped step index and are discarded; keeping the
  // chunks free of branches lets the independent draws interleave)
  float ea[NQ], eb[NQ];
  const int NT = (T + 31) >> 5;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    ea[i] = 0.0f;
    eb[i] = 0.0f;
    if (i < NT) {
      const int t = min(32 * i + c32, T - 1);
      draw_eps((uint32_t)t, (uint32_t)k, a.nk, ea[i], eb[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int t = 32 * i + c32;
    if (i < NT && t < T) {
      myE[2 * t] = ea[i];
      myE[2 * t + 1] = eb[i];
      if constexpr (kNetV) {
        // g(v) of the step (v = u + eps, or eps for an exploration sample), for the chain
        const float u0 = a.U[2 * t], u1 = a.U[2 * t + 1];
        myV[2 * t] = fminf(fmaxf(zm ? ea[i] : u0 + ea[i], a.u_lo0), a.u_hi0);
        myV[2 * t + 1] = fminf(fmaxf(zm ? eb[i] : u1 + eb[i], a.u_lo1), a.u_hi1);
      }
    }
  }
  if constexpr (MODEL == kModelBasis) {
    // the terms of each of the lane's steps that depend on the control alone:
    // {sin u_delta, -tan u_delta, u_delta, 0} and, per output o, Theta[1][o] u_F
    // + Theta[9][o] sin u_delta + Theta[24][o] u_F^2 + Theta[25][o] u_F^3
    float* myB = sB + slot * T * 8;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int t = 32 * i + c32;
      if (i < NT && t < T) {
        const float u0 = a.U[2 * t], u1 = a.U[2 * t + 1];
        const float vc0 = fminf(fmaxf(zm ? ea[i] : u0 + ea[i], a.u_lo0), a.u_hi0);
        const float vc1 = fminf(fmaxf(zm ? eb[i] : u1 + eb[i], a.u_lo1), a.u_hi1);
        const float sd = sinf(vc0);
        const float ntd = -tanf(vc0);
        const float u2 = vc1 * vc1, u3 = vc1 * u2;
        float c[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
          float acc = a.params[0 * 4 + o] * vc1;
          acc = __builtin_fmaf(a.params[8 * 4 + o], sd, acc);
          acc = __builtin_fmaf(a.params[23 * 4 + o], u2, acc);
          c[o] = __builtin_fmaf(a.params[24 * 4 + o], u3, acc);
        }
        *reinterpret_cast<float4*>(myB + 8 * t) = make_float4(sd, ntd, vc0, 0.0f);
        *reinterpret_cast<float4*>(myB + 8 * t + 4) = make_float4(c[0], c[1], c[2], c[3]);
      }
    }
  }
  Acc xd{x0v[3 + comp], 0.0f};       // NQ = 8: compensated in the chain
  float xh = x0v[3 + comp];           // NQ = 4: the uncompensated state hi_t
  if (c32 < 4) sX[slot * T4 * kXW + c32] = x0v[3 + c32];
  if (a.ckpt && valid && c32 < kStateDim)
    a.ckpt[(size_t)k * (T / a.ckpt_every + 1) * kCkptStride + c32] = x0v[c32];
  __syncthreads();

  // ---- B: serial chain of the dynamic states ---------------------------------------
  {
  float2 u = *reinterpret_cast<const float2*>(sU);
  float2 e = *reinterpret_cast<const float2*>(myE);
  float2 vc = make_float2(0.0f, 0.0f);
  if constexpr (kNetV) vc = *reinterpret_cast<const float2*>(myV);
  // the lane's store slot in sX: hi_{t+1} (lanes with bit 2 clear) or y_t (bit 2 set)
  const int xs_off = slot * T4 * kXW + ((lane & 4) ? 4 + comp : kXW + comp);
  // basis model: this step's control terms, also read one step ahead
  const float* myB = sB + slot * T * 8;
  float4 bq = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  float cq = 0.0f;
  if constexpr (MODEL == kModelBasis) {
    bq = *reinterpret_cast<const float4*>(myB);
    cq = myB[4 + comp];
  }
  for (int t = 0; t < T; ++t) {
    // next step's control and noise are read one step ahead (LDS latency off the chain)
    const int tn = min(t + 1, T - 1);
    float2 u_next = u, e_next = e, vc_next = vc;
    if constexpr (kNetV) {
      vc_next = *reinterpret_cast<const float2*>(myV + 2 * tn);
    } else {
      u_next = *reinterpret_cast<const float2*>(sU + 2 * tn);
      e_next = *reinterpret_cast<const float2*>(myE + 2 * tn);
    }
    const float vc0 = vc.x, vc1 = vc.y;
    float y;   // dt * f of the lane's component
    const float xcur = kDefer ? xh : xd.hi;
    if constexpr (MODEL == kModelBasis) {
      // bq = {sin u_delta, -tan u_delta, u_delta, 0}, cq = the control-only terms
      const float4 bq_next = *reinterpret_cast<const float4*>(myB + 8 * tn);
      const float cq_next = myB[8 * tn + 4 + comp];
      const float roll = dpp_f<0x00>(xcur), vx = dpp_f<0x55>(xcur);   // quad_perm:[i,i,i,i]
      const float vy = dpp_f<0xAA>(xcur), om = dpp_f<0xFF>(xcur);
      // tyre tangents: tan(arctan z) = z above v_x = 0.1, the steering alone below
      const bool mv = vx > 0.1f;
      const float rv = __builtin_amdgcn_rcpf(vx);
      const float q = vy * rv, w = om * rv;
      const float tf = mv ? __builtin_fmaf(0.45f, w, q) - bq.z : bq.y;
      const float tr = mv ? __builtin_fmaf(-0.35f, w, q) : 0.0f;
      const float qq = mv ? q : 0.0f;
      const float sf = bq.x * tf, tf2 = tf * tf, tr2 = tr * tr;
      const float atf = fabsf(tf), atr = fabsf(tr);
      const float rx = roll * vx, vx2 = vx * vx;
      const float raw[kRaw] = {vx, sf, sf * atf, sf * tf2, om * vy, om, vy, qq, tf, tf * atf, tf * tf2,
                               tr, tr * atr, tr * tr2, om * vx, roll, roll * om, rx, rx * om, vx2, vx * vx2};
      float p0 = cq, p1 = 0.0f, p2 = 0.0f, p3 = 0.0f;
#pragma unroll
      for (int i = 0; i < kRaw; i += 4) {
        p0 = __builtin_fmaf(kc[i], raw[i], p0);
        if (i + 1 < kRaw) p1 = __builtin_fmaf(kc[i + 1], raw[i + 1], p1);
        if (i + 2 < kRaw) p2 = __builtin_fmaf(kc[i + 2], raw[i + 2], p2);
        if (i + 3 < kRaw) p3 = __builtin_fmaf(kc[i + 3], raw[i + 3], p3);
      }
      y = a.dt * ((p0 + p1) + (p2 + p3));
      bq = bq_next;
      cq = cq_next;
    } else {
      // layer 1
      float acc1 = __builtin_fmaf(w1[4], vc0, bb1);
      acc1 = __builtin_fmaf(w1[5], vc1, acc1);
      // one asm block, so that no wait states are inserted between the four; the DPP
      // source xcur was written before this step's two fmas of acc1 above, the two wait
      // states a DPP read of a VALU result needs
      asm volatile(
          "v_fmac_f32_dpp %0, %1, %2 quad_perm:[0,0,0,0] row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %0, %1, %3 quad_perm:[1,1,1,1] row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %0, %1, %4 quad_perm:[2,2,2,2] row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %0, %1, %5 quad_perm:[3,3,3,3] row_mask:0xf bank_mask:0xf"
          : "+v"(acc1) : "v"(xcur), "v"(w1[0]), "v"(w1[1]), "v"(w1[2]), "v"(w1[3]));
      const float h1 = tanh_prescaled(acc1);
      // layer 2: four interleaved chains (P, Q for even and odd rotations) so that no
      // accumulator is read by the instruction right after the one that wrote it
      float P = __builtin_fmaf(wP[0], h1, bP);
      float Q = __builtin_fmaf(wQ[0], h1, bQ);
      float P2 = wP[1] * dpp_f<kRowRor + 1>(h1);
      float Q2 = wQ[1] * dpp_f<kRowRor + 1>(h1);
      // rotations 2..15 in one asm block (no wait states inserted between them); the
      // DPP source h1 was written before the four instructions forming P, Q, P2 and Q2,
      // which are the block's inputs: more than the two wait states a DPP read needs
      asm volatile(
          "v_fmac_f32_dpp %0, %4, %5 row_ror:2 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %1, %4, %6 row_ror:2 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %2, %4, %7 row_ror:3 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %3, %4, %8 row_ror:3 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %0, %4, %9 row_ror:4 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %1, %4, %10 row_ror:4 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %2, %4, %11 row_ror:5 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %3, %4, %12 row_ror:5 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %0, %4, %13 row_ror:6 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %1, %4, %14 row_ror:6 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %2, %4, %15 row_ror:7 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %3, %4, %16 row_ror:7 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %0, %4, %17 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %1, %4, %18 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %2, %4, %19 row_ror:9 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %3, %4, %20 row_ror:9 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %0, %4, %21 row_ror:10 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %1, %4, %22 row_ror:10 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %2, %4, %23 row_ror:11 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %3, %4, %24 row_ror:11 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %0, %4, %25 row_ror:12 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %1, %4, %26 row_ror:12 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %2, %4, %27 row_ror:13 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %3, %4, %28 row_ror:13 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %0, %4, %29 row_ror:14 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %1, %4, %30 row_ror:14 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %2, %4, %31 row_ror:15 row_mask:0xf bank_mask:0xf\n\t"
          "v_fmac_f32_dpp %3, %4, %32 row_ror:15 row_mask:0xf bank_mask:0xf"
          : "+v"(P), "+v"(Q), "+v"(P2), "+v"(Q2)
          : "v"(h1), "v"(wP[2]), "v"(wQ[2]), "v"(wP[3]), "v"(wQ[3]), "v"(wP[4]), "v"(wQ[4]), "v"(wP[5]), "v"(wQ[5]), "v"(wP[6]), "v"(wQ[6]), "v"(wP[7]), "v"(wQ[7]), "v"(wP[8]), "v"(wQ[8]), "v"(wP[9]), "v"(wQ[9]), "v"(wP[10]), "v"(wQ[10]), "v"(wP[11]), "v"(wQ[11]), "v"(wP[12]), "v"(wQ[12]), "v"(wP[13]), "v"(wQ[13]), "v"(wP[14]), "v"(wQ[14]), "v"(wP[15]), "v"(wQ[15]));
      P = P + P2;
      Q = Q + Q2;
      swap_rows(P, Q);                    // row 0: (P0, P1) -> out c;  row 1: (Q0, Q1) -> out 16+c
      const float h2 = tanh_prescaled(P + Q);
      // layer 3 (times dt): reduce-scatter of the four outputs over each quad, then the
      // quads of the row and the two rows
      const float A = __builtin_fmaf(wKA, h2, bKA) + dpp_f<kQuadXor1>(wSA * h2);   // output oA, lanes L, L^1
      const float B = wKB * h2 + dpp_f<kQuadXor1>(wSB * h2);                         // output oB, lanes L, L^1
      float g = A + dpp_f<kQuadXor2>(B);                                             // output oA, the quad
      g = g + dpp_f<kRowRor + 8>(g);
      g = g + dpp_f<kRowRor + 4>(g);
      y = add_rows(g);
    }
    // every lane of a component holds the same bits (y and the update are formed alike
    // in all of them), so all lanes store: no branch in the step loop
    if constexpr (kDefer) {
      xh = xh + y;
      sX[xs_off + t * kXW] = (lane & 4) ? y : xh;   // y_t at entry t, hi_{t+1} at entry t + 1
    } else {
      xd.add(y);
      sX[slot * T4 * kXW + (t + 1) * kXW + comp] = xd.value();
    }
    u = u_next;
    e = e_next;
    vc = vc_next;
  }
  }
  __syncthreads();

  // ---- C: kinematics and cost, parallel over t ---------------------------------------
  // Lane c owns the contiguous steps [c*npl, (c+1)*npl).  theta(t) = theta_0 + dt sum_{s<t}
  // theta_dot(s) and p(t+1) = p_0 + dt sum_{s<=t} R(theta(s)) v(s) are formed as
  // compensated lane sums plus compensated exclusive scans across the 32 lanes.  The
  // positions of all the lane's steps are formed first, then every map and decay load
  // is issued before the first is used (one memory round trip), then the costs.
  const int npl = NT;
  const int tb = c32 * npl;
  // x_d at the lane's steps, xv[q] = x_d(tb + q) for q = 0..NQ (the state before step
  // tb + q and after step tb + q - 1).  Deferred layout: x_d(t) = hi_t + lo_t, where lo_t
  // sums the rounding errors err_s = (hi_s + y_s) - fl(hi_s + y_s), s < t (error-free
  // two-sum), in the lane and then by a scan across the lanes; the chain's own sums
  // hi_{s+1} = fl(hi_s + y_s) are recomputed here.
  float4 xv[NQ + 1];
  if constexpr (kDefer) {
    float4 hv[NQ], yv[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int t = tb + q;
      const bool live = q < npl && t < T;
      hv[q] = live ? myX[2 * t] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      yv[q] = live ? myX[2 * t + 1] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    float hs[NQ][4], lq[NQ][4];
    float lsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const float hq[4] = {hv[q].x, hv[q].y, hv[q].z, hv[q].w};
      const float yq[4] = {yv[q].x, yv[q].y, yv[q].z, yv[q].w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float e_;
        two_sum(hq[c], yq[c], hs[q][c], e_);
        lsum[c] = lsum[c] + e_;
        lq[q][c] = lsum[c];
      }
    }
    float pre[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) pre[c] = scan32_excl(lsum[c], c32);
    xv[0] = make_float4(hv[0].x + pre[0], hv[0].y + pre[1], hv[0].z + pre[2], hv[0].w + pre[3]);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      xv[q + 1] = make_float4(hs[q][0] + (pre[0] + lq[q][0]), hs[q][1] + (pre[1] + lq[q][1]),
                              hs[q][2] + (pre[2] + lq[q][2]), hs[q][3] + (pre[3] + lq[q][3]));
  }
  auto xpre = [&](int q) -> float4 {   // x_d before step tb + q
    if constexpr (kDefer) return xv[q]; else return myX[tb + q];
  };
  auto xpost = [&](int q) -> float4 {  // x_d after step tb + q
    if constexpr (kDefer) return xv[q + 1]; else return myX[tb + q + 1];
  };
  float th_h = 0.0f, th_l = 0.0f;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = tb + q;
    if (q < npl && t < T) {
      float s_, e_;
      two_sum(th_h, a.dt * xpre(q).w, s_, e_);
      th_h = s_;
      th_l += e_;
    }
  }
  scan32_excl2(th_h, th_l, c32);
  {
    float s_, e_;
    two_sum(x0v[2], th_h, s_, e_);
    th_h = s_;
    th_l = th_l + e_;
  }
  // theta at the lane's first step; walk the steps for the position increments
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
        const float4 xs = xpre(q);
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
  scan32_excl2(px_h, px_l, c32);
  scan32_excl2(py_h, py_l, c32);
  {
    float s_, e_;
    two_sum(x0v[0], px_h, s_, e_);
    px_h = s_;
    px_l += e_;
    two_sum(x0v[1], py_h, s_, e_);
    py_h = s_;
    py_l += e_;
  }
  // post-step poses of the lane's steps (dead slots keep the last live pose)
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
        two_sum(th, a.dt * xpre(q).w, s_, e_);
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
  // all gathers at once (indices are clamped to the map, steps to [1, T])
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
      const float4 xn = xpost(q);
      const float px1 = pxh[q] + pxl[q], py1 = pyh[q] + pyl[q];
      if (a.ckpt && ((t + 1) % a.ckpt_every) == 0 && valid) {
        float* cp = a.ckpt + ((size_t)k * (T / a.ckpt_every + 1) + (t + 1) / a.ckpt_every) * kCkptStride;
        cp[0] = px1; cp[1] = py1; cp[2] = th1[q];
        cp[3] = xn.x; cp[4] = xn.y; cp[5] = xn.z; cp[6] = xn.w;
      }
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
  sum32_2(S_h, S_l);
  float S = S_h + S_l;
  const bool okc = all32(ok);
  if (!valid || !okc || !finite_f(S)) S = kInf;
  if (valid && c32 == 0) store_through(a.S + k, S);   // read by the host or Algorithm 3's update

  if (a.cem_zeta > 0) {
    // Algorithm 3: the sample's delta row, for the elite average
    if (valid) {
      float* drow = a.D + (size_t)k * 2 * T;
      for (int o = c32; o < 2 * T; o += 32) drow[o] = zm ? myE[o] - sU[o] : myE[o];
    }
    return;   // the cross-entropy update runs in the launch that follows
  }

  // ---- D: softmin partial of the block's samples ------------------------------------
  const float wmin = fminf(S, other_half(S));
  if (lane == 0) scratch[wv] = wmin;
  __syncthreads();
  const float rho = fminf(fminf(scratch[0], scratch[1]), fminf(scratch[2], scratch[3]));
  const float e = rel_weight(S, rho, a.inv_lambda);
  const float epair = e + other_half(e);
  if (lane == 0) scratch[4 + wv] = epair;
  const int eStrideRed = eStride;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    if (i < NT) {
      const int t = 32 * i + c32;
      const int tc = min(t, T - 1);
      const float d0 = zm ? ea[i] - sU[2 * tc] : ea[i];
      const float d1 = zm ? eb[i] - sU[2 * tc + 1] : eb[i];
      const float n0 = e * d0, n1 = e * d1;
      const float p0 = n0 + other_half(n0);
      const float p1 = n1 + other_half(n1);
      if (half == 0 && t < T) {
        red[wv * eStrideRed + 2 * t] = p0;
        red[wv * eStrideRed + 2 * t + 1] = p1;
      }
    }
  }
  __syncthreads();
  float* N_lds = sE;   // the noise rows are no longer read
  for (int o = threadIdx.x; o < 2 * T; o += kWaveBlock)
    N_lds[o] = ((red[o] + red[eStrideRed + o]) + red[2 * eStrideRed + o]) + red[3 * eStrideRed + o];
  const float eta = ((scratch[4] + scratch[5]) + scratch[6]) + scratch[7];
  finish_iteration<kWaveBlock, MODEL, true, HID>(a, blockIdx.x, rho, eta, N_lds, red);
}

template __global__ void rollout_wave_kernel<32, 4, kModelNet>(RolloutArgs);
template __global__ void rollout_wave_kernel<32, 8, kModelNet>(RolloutArgs);
template __global__ void rollout_wave_kernel<32, 4, kModelBasis>(RolloutArgs);
template __global__ void rollout_wave_kernel<32, 8, kModelBasis>(RolloutArgs);

// Dynamic LDS bytes the wave kernel needs for horizon T.
// (The layout of the kernel's LDS: the deferred-compensation layout up to T = 128,
// where launch_wave picks NQ = 4.)
size_t wave_smem_bytes(int T, int model) {
  const size_t e = (size_t)((2 * T + 3) & ~3);
  const size_t T4 = (size_t)((T + 4) & ~3);
  const bool defer = T <= 128;
  const size_t v = model == kModelNet ? (size_t)kWaveSlots * e : 0;
  const size_t x = (size_t)kWaveSlots * T4 * (defer ? 8 : 4);
  const size_t red = defer ? 0 : 4 * e;
  const size_t basis = model == kModelBasis ? (size_t)kWaveSlots * T * 8 : 0;
  return sizeof(float) * (e + kWaveSlots * e + v + x + red + 16 + basis);
}

}  // namespace mppi
