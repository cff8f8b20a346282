// Rollout schedule "lane": one wavefront lane per sample.
//
// Every lane carries its sample's full state through the T-step loop in
// registers (Algorithm 1's inner loop), drawing eps from Philox on the fly.  The
// network weights are read with wave-uniform addresses, so the compiler serves
// them from the scalar cache into SGPR operands; the nominal controls sit in
// LDS.  This is the throughput schedule for large K: one sample per lane keeps
// every lane busy without cross-lane traffic.
#include "kernels_common.hip.h"

namespace mppi {

constexpr int kLaneBlock = 256;
constexpr int kLaneWaves = kLaneBlock / 64;

template <int HID>
__device__ __forceinline__ void net_forward_uniform(const float* __restrict__ P, const float in[6],
                                                    float f[4]) {
  const float* W1 = P;
  const float* b1 = W1 + HID * 6;
  const float* W2 = b1 + HID;
  const float* b2 = W2 + HID * HID;
  const float* W3 = b2 + HID;
  const float* b3 = W3 + 4 * HID;
  float h1[HID];
#pragma unroll
  for (int i = 0; i < HID; ++i) {
    float a = b1[i];
#pragma unroll
    for (int j = 0; j < 6; ++j) a = __builtin_fmaf(W1[i * 6 + j], in[j], a);
    h1[i] = tanh_f(a);
  }
  float h2[HID];
#pragma unroll
  for (int i = 0; i < HID; ++i) {
    float a = b2[i];
#pragma unroll
    for (int j = 0; j < HID; ++j) a = __builtin_fmaf(W2[i * HID + j], h1[j], a);
    h2[i] = tanh_f(a);
  }
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    float a = b3[o];
#pragma unroll
    for (int j = 0; j < HID; ++j) a = __builtin_fmaf(W3[o * HID + j], h2[j], a);
    f[o] = a;
  }
}

// Writes this block's (rho_g, eta_g, N_g[T][2]) by regenerating eps.
__device__ __forceinline__ void lane_block_partial(const RolloutArgs& a, float S, bool valid, int k,
                                                   float* red /* [kLaneWaves][2*kTMax] */,
                                                   float* scratch) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const float sv = valid ? S : kInf;
  const float rho = block_min<kLaneWaves>(sv, scratch);
  const float e = rel_weight(sv, rho, a.inv_lambda);
  const float eta = block_sum<kLaneWaves>(e, scratch);
  for (int t = 0; t < a.T; ++t) {
    float e0 = 0.0f, e1 = 0.0f;
    if (valid) draw_eps((uint32_t)t, (uint32_t)k, a.nk, e0, e1);
    const float n0 = wave_sum(e * e0);
    const float n1 = wave_sum(e * e1);
    if (lane == 0) {
      red[w * 2 * kTMax + 2 * t] = n0;
      red[w * 2 * kTMax + 2 * t + 1] = n1;
    }
  }
  __syncthreads();
  const int stride = 2 + 2 * a.T;
  float* out = a.part + (size_t)blockIdx.x * stride;
  for (int o = threadIdx.x; o < 2 * a.T; o += kLaneBlock) {
    float s = red[o];
#pragma unroll
    for (int i = 1; i < kLaneWaves; ++i) s += red[i * 2 * kTMax + o];
    out[2 + o] = s;
  }
  if (threadIdx.x == 0) {
    out[0] = rho;
    out[1] = eta;
  }
}

template <int HID>
__global__ __launch_bounds__(kLaneBlock) void rollout_lane_kernel(RolloutArgs a) {
  __shared__ float sU[2 * kTMax];
  __shared__ float red[kLaneWaves * 2 * kTMax];
  __shared__ float scratch[kLaneWaves];
  for (int i = threadIdx.x; i < 2 * a.T; i += kLaneBlock) sU[i] = a.U[i];
  __syncthreads();
  const int k = blockIdx.x * kLaneBlock + threadIdx.x;
  const bool valid = k < a.K;
  // state and cost in compensated form (hi + lo); the network and the kinematics
  // read the hi parts, the cost reads hi + lo
  Acc x[kStateDim];
#pragma unroll
  for (int i = 0; i < kStateDim; ++i) {
    x[i].hi = a.x0_dev ? a.x0_dev[i] : a.x0[i];
    x[i].lo = 0.0f;
  }
  Acc S{0.0f, 0.0f};
  bool ok = true;
  float Sv = kInf;
  if (valid) {
    for (int t = 0; t < a.T; ++t) {
      float e0, e1;
      draw_eps((uint32_t)t, (uint32_t)k, a.nk, e0, e1);
      const float u0 = sU[2 * t], u1 = sU[2 * t + 1];
      const float vc0 = fminf(fmaxf(u0 + e0, a.u_lo0), a.u_hi0);
      const float vc1 = fminf(fmaxf(u1 + e1, a.u_lo1), a.u_hi1);
      const float in[6] = {x[3].hi, x[4].hi, x[5].hi, x[6].hi, vc0, vc1};
      float f[4];
      net_forward_uniform<HID>(a.params, in, f);
      float sth, cth;
      sincosf(x[2].hi, &sth, &cth);
      const float dpx = a.dt * (cth * x[4].hi - sth * x[5].hi);
      const float dpy = a.dt * (sth * x[4].hi + cth * x[5].hi);
      const float dth = a.dt * x[6].hi;
      x[0].add(dpx);
      x[1].add(dpy);
      x[2].add(dth);
#pragma unroll
      for (int i = 0; i < 4; ++i) x[3 + i].add(a.dt * f[i]);
#pragma unroll
      for (int i = 0; i < kStateDim; ++i) ok = ok && finite_f(x[i].hi);
      S.add(state_cost2(a.cost, a.map, a.decay, x[0].hi, x[0].lo, x[1].hi, x[1].lo, x[4].value(),
                        x[5].value(), t + 1));
      S.add(a.gcs0 * (u0 * e0) + a.gcs1 * (u1 * e1));
    }
    Sv = S.value();
    if (!ok || !finite_f(Sv)) Sv = kInf;
    a.S[k] = Sv;
  }
  lane_block_partial(a, Sv, valid, k, red, scratch);
  finish_iteration<kLaneBlock>(a, red);
}

template __global__ void rollout_lane_kernel<32>(RolloutArgs);
template __global__ void rollout_lane_kernel<64>(RolloutArgs);

}  // namespace mppi
