// Shift, plant step and the stand-alone noise generator.  (Algorithm 2's weights and
// the update of U run at the end of the rollout kernels, see finish_iteration.)
#include "kernels_common.hip.h"

namespace mppi {

// Algorithm 1's last block: u0_out = u_0; u_{t-1} <- u_t; u_{T-1} <- Initialize = (0,0).
__global__ __launch_bounds__(512) void shift_kernel(float* U, int T, float* u0_out) {
  const int o = threadIdx.x;
  float v = 0.0f;
  if (o + 2 < 2 * T) v = U[o + 2];
  if (o < 2 && u0_out) u0_out[o] = U[o];
  __syncthreads();
  if (o < 2 * T) U[o] = v;
}

// Noise-free plant step x_out = F(x, g(u)) with the FP32 network, or with the
// basis-function model when HID = 0 (one thread).
// x_out may alias x_in; x_copy (nullable) receives a second copy of the result.
template <int HID>
__global__ void plant_kernel(const float* __restrict__ P, const float* x_in, const float* u,
                             float* x_out, float* x_copy, float dt, float lo0, float lo1, float hi0,
                             float hi1) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float x[kStateDim];
  for (int i = 0; i < kStateDim; ++i) x[i] = x_in[i];
  const float vc0 = fminf(fmaxf(u[0], lo0), hi0);
  const float vc1 = fminf(fmaxf(u[1], lo1), hi1);
  const float in[6] = {x[3], x[4], x[5], x[6], vc0, vc1};
  float f[4];
  if constexpr (HID == 0) {
    basis_f(P, in, vc0, vc1, f);
  } else {
    const float* W1 = P;
    const float* b1 = W1 + HID * 6;
    const float* W2 = b1 + HID;
    const float* b2 = W2 + HID * HID;
    const float* W3 = b2 + HID;
    const float* b3 = W3 + 4 * HID;
    float h1[HID], h2[HID];
    for (int i = 0; i < HID; ++i) {
      float acc = b1[i];
      for (int j = 0; j < 6; ++j) acc = __builtin_fmaf(W1[i * 6 + j], in[j], acc);
      h1[i] = tanh_f(acc);
    }
    for (int i = 0; i < HID; ++i) {
      float acc = b2[i];
      for (int j = 0; j < HID; ++j) acc = __builtin_fmaf(W2[i * HID + j], h1[j], acc);
      h2[i] = tanh_f(acc);
    }
    for (int o = 0; o < 4; ++o) {
      float acc = b3[o];
      for (int j = 0; j < HID; ++j) acc = __builtin_fmaf(W3[o * HID + j], h2[j], acc);
      f[o] = acc;
    }
  }
  float sth, cth;
  sincosf(x[2], &sth, &cth);
  float y[kStateDim];
  y[0] = x[0] + dt * (cth * x[4] - sth * x[5]);
  y[1] = x[1] + dt * (sth * x[4] + cth * x[5]);
  y[2] = x[2] + dt * x[6];
  for (int i = 0; i < 4; ++i) y[3 + i] = x[3 + i] + dt * f[i];
  for (int i = 0; i < kStateDim; ++i) {
    x_out[i] = y[i];
    if (x_copy) x_copy[i] = y[i];
  }
}

template __global__ void plant_kernel<0>(const float*, const float*, const float*, float*, float*,
                                         float, float, float, float, float);
template __global__ void plant_kernel<32>(const float*, const float*, const float*, float*, float*,
                                          float, float, float, float, float);
template __global__ void plant_kernel<64>(const float*, const float*, const float*, float*, float*,
                                          float, float, float, float, float);

// The cost map h at n world positions xy[n][2], with the rollout kernels' interpolation.
__global__ __launch_bounds__(256) void costmap_kernel(CostArgs c, const float* __restrict__ map,
                                                      const float* __restrict__ xy, int n, float* h) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  h[i] = costmap_at2(c, map, xy[2 * i], 0.0f, xy[2 * i + 1], 0.0f);
}

// The rollout kernels' perturbations for one iteration, written out ([K][T][2]).
__global__ __launch_bounds__(256) void noise_kernel(NoiseKey nk, int K, int T, float* eps) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= K * T) return;
  const int k = idx / T, t = idx - k * T;
  float e0, e1;
  draw_eps((uint32_t)t, (uint32_t)k, nk, e0, e1);
  eps[2 * (size_t)idx] = e0;
  eps[2 * (size_t)idx + 1] = e1;
}

// K-shard merge: the n partial rows (rho_g, eta_g, N_g[T][2]) that the shards of one
// iteration exported are merged exactly as the blocks of one launch are (Algorithm 2:
// rho = min_g rho_g, eta~ = sum_g exp(-(rho_g - rho)/lambda) eta_g, Delta = the same
// combination of the N_g over eta~), then smoothed and applied to U, with the statistics
// and the status, by the final stage of the rollout kernels.  One block.
__global__ __launch_bounds__(256) void merge_update_kernel(RolloutArgs a, const float* rows, int n) {
  __shared__ float lds[2 * kTMax];
  __shared__ float s_small[2 * kMergeChunk];
  FinalStage<256, kModelNet, false> fs;
  fs.prefetch(a);
  float rho, eta;
  merge_rows<256>(rows, n, 2 + 2 * a.T, 2 * a.T, a.inv_lambda, lds, s_small, rho, eta);
  __syncthreads();
  const bool fin = (rho < kInf) && (eta > 0.0f);
  fs.apply(a, lds, fin, fin ? 1.0f / eta : 0.0f, a.params, rho, fin ? eta : 0.0f, a.nk.iter, a.u0_out, a.x_copy);
}

}  // namespace mppi
