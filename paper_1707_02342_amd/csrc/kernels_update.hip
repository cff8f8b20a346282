// Weights, update, shift, plant step and the stand-alone noise generator.
//
// merge_update_kernel: Algorithm 2 and the update line of Algorithm 1 from the
// rollout blocks' partials.  One workgroup: rho = min_g rho_g; per-block scale
// s_g = exp(-(rho_g - rho)/lambda); eta~ = sum_g s_g eta_g; Delta_t = sum_g s_g N_g[t] / eta~;
// U_t += sum_j SG[t][j] Delta_j.  If no sample had a finite cost the status is
// NONFINITE and U is left unchanged (the shift of Section III-D-1 guarantees a
// non-zero weight otherwise).
#include "kernels_common.hip.h"

namespace mppi {

constexpr int kMergeBlock = 512;
constexpr int kMergeWaves = kMergeBlock / 64;
constexpr int kNonfinite = 5;

__global__ __launch_bounds__(kMergeBlock) void merge_update_kernel(MergeArgs a, float* scale) {
  __shared__ float scratch[kMergeWaves];
  __shared__ float s_delta[2 * kTMax];
  const int stride = 2 + 2 * a.T;
  float m = kInf;
  for (int g = threadIdx.x; g < a.G; g += kMergeBlock) m = fminf(m, a.part[(size_t)g * stride]);
  const float rho = block_min<kMergeWaves>(m, scratch);
  float es = 0.0f;
  for (int g = threadIdx.x; g < a.G; g += kMergeBlock) {
    const float rg = a.part[(size_t)g * stride];
    const float eg = a.part[(size_t)g * stride + 1];
    const float sc = (eg > 0.0f) ? expf(-(rg - rho) * a.inv_lambda) : 0.0f;
    scale[g] = sc;
    es = __builtin_fmaf(sc, eg, es);
  }
  const float eta = block_sum<kMergeWaves>(es, scratch);
  if (!(rho < kInf) || !(eta > 0.0f)) {
    if (threadIdx.x == 0) {
      *a.status = kNonfinite;
      a.stats[0] = rho;
      a.stats[1] = 0.0f;
    }
    for (int o = threadIdx.x; o < 2 * a.T; o += kMergeBlock) a.stats[2 + o] = 0.0f;
    return;
  }
  __syncthreads();   // scale[] written by other threads
  const float inv_eta = 1.0f / eta;
  for (int o = threadIdx.x; o < 2 * a.T; o += kMergeBlock) {
    float acc = 0.0f;
    for (int g = 0; g < a.G; ++g) acc = __builtin_fmaf(scale[g], a.part[(size_t)g * stride + 2 + o], acc);
    const float d = acc * inv_eta;
    s_delta[o] = d;
    a.stats[2 + o] = d;
  }
  __syncthreads();
  const int w = a.sg_window;
  if (!a.update_U) {
    if (threadIdx.x == 0) {
      *a.status = 0;
      a.stats[0] = rho;
      a.stats[1] = eta;
    }
    return;
  }
  for (int o = threadIdx.x; o < 2 * a.T; o += kMergeBlock) {
    float upd;
    if (w == 1) {
      upd = s_delta[o];
    } else {
      const int t = o >> 1, c = o & 1;
      const int lo = min(max(t - w / 2, 0), a.T - w);
      const float* row = a.sg + (size_t)t * w;
      upd = 0.0f;
      for (int j = 0; j < w; ++j) upd = __builtin_fmaf(row[j], s_delta[2 * (lo + j) + c], upd);
    }
    a.U[o] = a.U[o] + upd;
  }
  if (threadIdx.x == 0) {
    *a.status = 0;
    a.stats[0] = rho;
    a.stats[1] = eta;
  }
}

// Algorithm 1's last block: u0_out = u_0; u_{t-1} <- u_t; u_{T-1} <- Initialize = (0,0).
__global__ __launch_bounds__(512) void shift_kernel(float* U, int T, float* u0_out) {
  const int o = threadIdx.x;
  float v = 0.0f;
  if (o + 2 < 2 * T) v = U[o + 2];
  if (o < 2 && u0_out) u0_out[o] = U[o];
  __syncthreads();
  if (o < 2 * T) U[o] = v;
}

// Noise-free plant step x_out = F(x, g(u)) with the FP32 network (one thread).
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
  const float* W1 = P;
  const float* b1 = W1 + HID * 6;
  const float* W2 = b1 + HID;
  const float* b2 = W2 + HID * HID;
  const float* W3 = b2 + HID;
  const float* b3 = W3 + 4 * HID;
  float h1[HID], h2[HID], f[4];
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

template __global__ void plant_kernel<32>(const float*, const float*, const float*, float*, float*,
                                          float, float, float, float, float);
template __global__ void plant_kernel<64>(const float*, const float*, const float*, float*, float*,
                                          float, float, float, float, float);

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

}  // namespace mppi
