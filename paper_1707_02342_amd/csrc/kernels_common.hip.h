// Reductions and the per-block softmin partial shared by the rollout kernels.
//
// Each rollout block ends by summarising its samples as
//   rho_g = min_k S_k,  eta_g = sum_k exp(-(S_k - rho_g)/lambda),
//   N_g[t] = sum_k exp(-(S_k - rho_g)/lambda) eps_{k,t}
// so that the merge kernel can form Algorithm 2's weights and the weighted
// perturbation sum exactly: rho = min_g rho_g, eta~ = sum_g e^{-(rho_g-rho)/lambda} eta_g,
// Delta_t = sum_g e^{-(rho_g-rho)/lambda} N_g[t] / eta~.  All sums run in a fixed
// order, so results are reproducible run to run.
#pragma once

#include "device_common.h"

namespace mppi {

constexpr float kInf = __builtin_huge_valf();

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fminf(v, __shfl_xor(v, m, 64));
  return v;
}

// Block-wide min / sum over NW waves through LDS, result in every lane.
template <int NW>
__device__ __forceinline__ float block_min(float v, float* scratch) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_min(v);
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  float r = scratch[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) r = fminf(r, scratch[i]);
  __syncthreads();
  return r;
}

template <int NW>
__device__ __forceinline__ float block_sum(float v, float* scratch) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  float r = scratch[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) r += scratch[i];
  __syncthreads();
  return r;
}

// Unnormalised weight of a sample relative to the block minimum.
__device__ __forceinline__ float rel_weight(float S, float rho, float inv_lambda) {
  return (S < kInf && rho < kInf) ? expf(-(S - rho) * inv_lambda) : 0.0f;
}

}  // namespace mppi
