// Reductions and the per-block softmin partial shared by the rollout kernels.
//
// Each rollout block ends by summarising its samples as
//   rho_g = min_k S_k,  eta_g = sum_k exp(-(S_k - rho_g)/lambda),
//   N_g[t] = sum_k exp(-(S_k - rho_g)/lambda) eps_{k,t}
// so that the last block to finish can form Algorithm 2's weights and the weighted
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

constexpr int kMergeChunk = 64;
constexpr int kStatusNonfinite = 5;

// Merge n partial rows (rho_g, eta_g, N_g[2T]) into one relative to rho = min_g rho_g:
// eta = sum_g s_g eta_g, N = sum_g s_g N_g, s_g = exp(-(rho_g - rho)/lambda) (s_g = 0 for
// a row without finite samples).  Called by the whole block.  Rows are taken in chunks
// of kMergeChunk whose scales are staged in LDS; every sum runs in row order, so the
// result does not depend on NT or on the chunking.  The result row goes to out_row
// (global) and/or out_lds.  T2 <= 2 * kTMax.
template <int NT>
__device__ void merge_rows(const float* rows, int n, int stride, int T2, float inv_lambda,
                           float* out_row, float* out_lds, float* s_small /* [2 * kMergeChunk] */,
                           float& rho_out, float& eta_out) {
  constexpr int kOut = (2 * kTMax + NT - 1) / NT;
  const int tid = threadIdx.x;
  float r = kInf;
  for (int g = tid; g < n; g += NT) r = fminf(r, __builtin_nontemporal_load(rows + (size_t)g * stride));
  const float rho = block_min<NT / 64>(r, s_small);
  float eta = 0.0f;
  float acc[kOut];
#pragma unroll
  for (int j = 0; j < kOut; ++j) acc[j] = 0.0f;
  for (int c0 = 0; c0 < n; c0 += kMergeChunk) {
    const int m = min(kMergeChunk, n - c0);
    if (tid < m) {
      const float* row = rows + (size_t)(c0 + tid) * stride;
      const float eg = __builtin_nontemporal_load(row + 1);
      s_small[tid] = (eg > 0.0f) ? expf(-(__builtin_nontemporal_load(row) - rho) * inv_lambda) : 0.0f;
      s_small[kMergeChunk + tid] = eg;
    }
    __syncthreads();
    for (int g = 0; g < m; ++g) eta = __builtin_fmaf(s_small[g], s_small[kMergeChunk + g], eta);
#pragma unroll
    for (int j = 0; j < kOut; ++j) {
      const int o = tid + j * NT;
      if (o < T2) {
        const float* col = rows + (size_t)c0 * stride + 2 + o;
        int g = 0;
        for (; g + 16 <= m; g += 16) {
          float v[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) v[i] = __builtin_nontemporal_load(col + (size_t)(g + i) * stride);
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[j] = __builtin_fmaf(s_small[g + i], v[i], acc[j]);
        }
        for (; g < m; ++g) acc[j] = __builtin_fmaf(s_small[g], __builtin_nontemporal_load(col + (size_t)g * stride), acc[j]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < kOut; ++j) {
    const int o = tid + j * NT;
    if (o < T2) {
      if (out_row) out_row[2 + o] = acc[j];
      if (out_lds) out_lds[o] = acc[j];
    }
  }
  if (tid == 0 && out_row) {
    out_row[0] = rho;
    out_row[1] = eta;
  }
  rho_out = rho;
  eta_out = eta;
}

// Called by every rollout block after writing its partial row (tile = the block's
// index among the launch's blocks of this problem).  Blocks arrive in groups of
// merge_group_size(G); the last to arrive in a group merges the group's rows, and the last group merger
// merges the group rows and applies Algorithm 2's normalisation, the Savitzky-Golay
// smoothing and the update U <- U + SG * Delta.  Device-scope fences order the rows
// written on one XCD before their reads on another.  Every decision is uniform over
// the block, so all barriers are reached by all threads.
template <int NT>
__device__ void finish_iteration(const RolloutArgs& a, int tile, float* lds /* >= 2T floats */) {
  __shared__ unsigned s_flag;
  __shared__ float s_small[2 * kMergeChunk];
  const int tid = threadIdx.x;
  const int T2 = 2 * a.T;
  const int stride = 2 + T2;
  const int gsz = merge_group_size(a.G);
  const int ngrp = (a.G + gsz - 1) / gsz;
  const int grp = tile / gsz;
  const int n_in = min(gsz, a.G - grp * gsz);
  __threadfence();
  __syncthreads();
  if (tid == 0) s_flag = (atomicAdd(a.cnt + grp, 1u) == (unsigned)(n_in - 1)) ? 1u : 0u;
  __syncthreads();
  if (s_flag) {
    __threadfence();
    float rho, eta;
    merge_rows<NT>(a.part + (size_t)grp * gsz * stride, n_in, stride, T2, a.inv_lambda,
                   a.part2 + (size_t)grp * stride, nullptr, s_small, rho, eta);
    if (tid == 0) a.cnt[grp] = 0u;
    __threadfence();
    __syncthreads();
    if (tid == 0) s_flag = (atomicAdd(a.cnt + ngrp, 1u) == (unsigned)(ngrp - 1)) ? 1u : 0u;
    __syncthreads();
    if (s_flag) {
      __threadfence();
      merge_rows<NT>(a.part2, ngrp, stride, T2, a.inv_lambda, nullptr, lds, s_small, rho, eta);
      if (tid == 0) a.cnt[ngrp] = 0u;
      const bool fin = (rho < kInf) && (eta > 0.0f);
      const float inv_eta = fin ? 1.0f / eta : 0.0f;
      for (int o = tid; o < T2; o += NT) {
        const float d = lds[o] * inv_eta;
        lds[o] = d;
        a.stats[2 + o] = d;
      }
      __syncthreads();
      if (fin && a.update_U) {
        const int w = a.sg_window;
        for (int o = tid; o < T2; o += NT) {
          float upd;
          if (w == 1) {
            upd = lds[o];
          } else {
            const int t = o >> 1, c = o & 1;
            const int lo = min(max(t - w / 2, 0), a.T - w);
            const float* row = a.sg + (size_t)t * w;
            upd = 0.0f;
            for (int j = 0; j < w; ++j) upd = __builtin_fmaf(row[j], lds[2 * (lo + j) + c], upd);
          }
          a.Uout[o] = a.Uout[o] + upd;
        }
      }
      if (tid == 0) {
        *a.status = fin ? 0 : kStatusNonfinite;
        a.stats[0] = rho;
        a.stats[1] = fin ? eta : 0.0f;
        if (a.iter_dev) *a.iter_dev = *a.iter_dev + 1u;
      }
    }
  }
  __syncthreads();
}

}  // namespace mppi
