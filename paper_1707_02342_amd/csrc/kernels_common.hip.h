// Reductions and the per-block softmin partial shared by the rollout kernels.
//
// Each rollout block ends by summarising its samples as
//   rho_g = min_k S_k,  eta_g = sum_k exp(-(S_k - rho_g)/lambda),
//   N_g[t] = sum_k exp(-(S_k - rho_g)/lambda) delta_{k,t},
// delta_{k,t} = v_{k,t} - u_t (eps_{k,t}, or eps_{k,t} - u_t for an exploration sample drawn
// around zero), so that the last block to finish can form Algorithm 2's weights and the weighted
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

// A store that writes through the XCD's L2 (device-scope relaxed atomic store).  Data
// that other blocks read in the same launch, and results read by the host, are
// written this way.
__device__ __forceinline__ void store_through(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A load that sees every store_through completed before it (device-scope relaxed
// atomic load: it does not return a stale line of the XCD's L2).
__device__ __forceinline__ float load_through(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The work queue of a persistent launch: queue[0] counts the work items handed out,
// queue[1] the blocks that have found the queue empty.  Returns the calling block's next
// item (the same in every thread), or -1 once all n_items have been handed out.  The
// last block to find the queue empty resets both words (every other block has taken its
// last item by then), so each launch, also one replayed from a captured graph, starts
// from zero without a memset.  Every block calls it until it returns -1.
__device__ __forceinline__ int next_work_item(unsigned* queue, int n_items) {
  __shared__ int s_item;
  __syncthreads();   // the block is done with its previous item
  if (threadIdx.x == 0) {
    int b = (int)atomicAdd(queue, 1u);
    if (b >= n_items) {
      b = -1;
      if (atomicAdd(queue + 1, 1u) == gridDim.x - 1u) {
        __hip_atomic_store(queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(queue + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    s_item = b;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s_item);   // uniform: the item's data is read with scalar loads
}

constexpr int kMergeChunk = 64;
constexpr int kStatusNonfinite = 5;

// Merge n partial rows (rho_g, eta_g, N_g[2T]) into one relative to rho = min_g rho_g:
// eta = sum_g s_g eta_g, N = sum_g s_g N_g, s_g = exp(-(rho_g - rho)/lambda) (s_g = 0 for
// a row without finite samples).  Called by the whole block.  Rows are taken in chunks
// of kMergeChunk whose scales are staged in LDS; every sum runs in row order, so the
// result does not depend on NT or on the chunking.  N goes to out_lds[2T] (visible to
// the block after its next barrier), rho and eta to every thread.  T2 <= 2 * kTMax.
template <int NT>
__device__ void merge_rows(const float* rows, int n, int stride, int T2, float inv_lambda,
                           float* out_lds, float* s_small /* [2 * kMergeChunk] */,
                           float& rho_out, float& eta_out) {
  constexpr int kOut = (2 * kTMax + NT - 1) / NT;
  constexpr int kFast = 16;
  static_assert(kMergeChunk >= kFast, "");
  const int tid = threadIdx.x;
  float acc[kOut];
#pragma unroll
  for (int j = 0; j < kOut; ++j) acc[j] = 0.0f;
  float rho, eta = 0.0f;
  if (n <= kFast) {
    // one round trip: every load of the n rows is issued before the first use
    float rg = kInf, eg = 0.0f;
    if (tid < n) {
      rg = load_through(rows + (size_t)tid * stride);
      eg = load_through(rows + (size_t)tid * stride + 1);
    }
    float v[kOut][kFast];
#pragma unroll
    for (int j = 0; j < kOut; ++j) {
      const int o = tid + j * NT;
#pragma unroll
      for (int g = 0; g < kFast; ++g)
        v[j][g] = (o < T2 && g < n) ? load_through(rows + (size_t)g * stride + 2 + o) : 0.0f;
    }
    if (tid < n) {
      s_small[tid] = rg;
      s_small[kMergeChunk + tid] = eg;
    }
    __syncthreads();
    rho = kInf;
    for (int g = 0; g < n; ++g) rho = fminf(rho, s_small[g]);
    __syncthreads();
    if (tid < n) s_small[tid] = (eg > 0.0f) ? expf(-(rg - rho) * inv_lambda) : 0.0f;
    __syncthreads();
    for (int g = 0; g < n; ++g) eta = __builtin_fmaf(s_small[g], s_small[kMergeChunk + g], eta);
#pragma unroll
    for (int j = 0; j < kOut; ++j)
#pragma unroll
      for (int g = 0; g < kFast; ++g)
        if (g < n) acc[j] = __builtin_fmaf(s_small[g], v[j][g], acc[j]);
    __syncthreads();
  } else {
    float r = kInf;
    for (int g = tid; g < n; g += NT) r = fminf(r, load_through(rows + (size_t)g * stride));
    rho = block_min<NT / 64>(r, s_small);
    for (int c0 = 0; c0 < n; c0 += kMergeChunk) {
      const int m = min(kMergeChunk, n - c0);
      if (tid < m) {
        const float* row = rows + (size_t)(c0 + tid) * stride;
        const float eg = load_through(row + 1);
        s_small[tid] = (eg > 0.0f) ? expf(-(load_through(row) - rho) * inv_lambda) : 0.0f;
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
            for (int i = 0; i < 16; ++i) v[i] = load_through(col + (size_t)(g + i) * stride);
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[j] = __builtin_fmaf(s_small[g + i], v[i], acc[j]);
          }
          for (; g < m; ++g)
            acc[j] = __builtin_fmaf(s_small[g], load_through(col + (size_t)g * stride), acc[j]);
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int j = 0; j < kOut; ++j) {
    const int o = tid + j * NT;
    if (o < T2) out_lds[o] = acc[j];
  }
  rho_out = rho;
  eta_out = eta;
}

// Wave 0 publishes a row (rho, eta, N[T2]) to global memory and counts its arrival
// at *cnt; returns, in every thread after the barrier, whether this block was the
// last of `expected` arrivals.  The row is written through L2, and the wave waits
// until those stores have completed (reached the device's point of coherence) before
// it counts, so the last block, which reads the rows with load_through after the
// count, sees every row.  This orders exactly the row's stores, where a device-scope
// release fence would also write back every dirty line of the XCD's L2, and the
// reads need no device-scope acquire (which would invalidate the L2).
// meanwhile() runs in every thread while the count is in flight (waves 1.. before the
// barrier, wave 0 once its atomic has been issued), so loads it makes overlap the
// count's round trip.
template <int NT, class Meanwhile>
__device__ bool publish_and_count(float* dst, float rho, float eta, const float* N_lds, int T2,
                                  unsigned* cnt, unsigned expected, unsigned* s_flag, Meanwhile&& meanwhile) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0) {
      store_through(dst, rho);
      store_through(dst + 1, eta);
    }
    for (int o = lane; o < T2; o += 64) store_through(dst + 2 + o, N_lds[o]);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    unsigned old = 0u;
    if (lane == 0) old = atomicAdd(cnt, 1u);
    meanwhile();
    if (lane == 0) *s_flag = (old == expected - 1u) ? 1u : 0u;
  } else {
    meanwhile();
  }
  __syncthreads();
  return *s_flag != 0u;
}

template <int NT>
__device__ bool publish_and_count(float* dst, float rho, float eta, const float* N_lds, int T2,
                                  unsigned* cnt, unsigned expected, unsigned* s_flag) {
  return publish_and_count<NT>(dst, rho, eta, N_lds, T2, cnt, expected, s_flag, [] {});
}

// The value of v in lane `src` of the calling wave (src uniform).
__device__ __forceinline__ float lane_value(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}

// The plant layout of the network's parameter vector (width H, a multiple of 4), the same
// number of floats: W1[H][6] and b1[H] in place, W2 as [H/4][H][4] (neuron n's weights
// 4q .. 4q+3 in one 16-byte word, the words of consecutive neurons consecutive), b2[H]
// in place, W3 as [H/4][4][4] (the same for the 4 outputs), b3[4] in place.  Returns
// where element i of the parameter vector (W1[H][6], b1, W2[H][H], b2, W3[4][H], b3) goes.
__host__ __device__ constexpr int plant_layout_index(int i, int H) {
  const int oW2 = 7 * H, oW3 = 8 * H + H * H;
  if (i >= oW2 && i < oW2 + H * H) {
    const int n = (i - oW2) / H, j = (i - oW2) % H;
    return oW2 + (((j >> 2) * H + n) << 2) + (j & 3);
  }
  if (i >= oW3 && i < oW3 + 4 * H) {
    const int o = (i - oW3) / H, j = (i - oW3) % H;
    return oW3 + (((j >> 2) * 4 + o) << 2) + (j & 3);
  }
  return i;   // W1 and the biases keep their places
}

// The receding-horizon part of a control step (Algorithm 1's last block and the
// plant), run by the final merge after the update: U is shifted (u_0 out,
// u_{t-1} <- u_t, u_{T-1} <- (0, 0)), and the plant state in x0_dev advances by one
// noise-free step x <- F(x, g(u_0)).  The plant step runs in wave 0 alone, without
// block barriers: the network one neuron per lane (the hidden width is at most 64), each
// neuron's sum in input order with the previous layer's outputs read lane by lane, so
// the new state equals a one-thread evaluation bit for bit.  x_lane: component tid of
// the plant state before the step (threads tid < 7), loaded by the merging block before
// its merge; every other block of the launch has read x0_dev before it published its
// row, so x0_dev can be overwritten here.  lds (>= 2T floats) holds Delta on entry,
// still read by the smoothing of other threads.
// MODEL: the dynamics model the calling kernel serves (kModelAny: decided by a.model);
// a kernel that serves one model compiles only that model's plant step.  HC: the
// network width when the calling kernel fixes it (0: a.hidden), so that every sum is
// unrolled and its weight loads issued together (the arithmetic is the same).
// writer = false: a block that runs the step only for itself (the multi-step launch's
// replicated final stage) writes nothing to global memory.  u_next, x_next (LDS,
// nullable): where the shifted U ([2T]) and the new plant state ([7]) also go; x_next is
// written by wave 0 and visible to the block after its next barrier.
// PL: params holds the network in the plant layout (plant_layout_index; HC > 0), whose
// weight reads are 16-byte words, consecutive over the lanes and independent of the sums.
template <int NT, int kOut, int MODEL, int HC = 0, bool PL = false>
__device__ void receding_step(const RolloutArgs& a, const float (&u_new)[kOut], float x_lane, float* lds,
                              const float* params, float* u0_out, float* x_copy, bool writer = true,
                              float* u_next = nullptr, float* x_next = nullptr) {
  constexpr bool kMayBasis = MODEL != kModelNet;
  constexpr bool kMayNet = MODEL != kModelBasis;
  __shared__ float s_x[kStateDim];
  const int tid = threadIdx.x;
  const int T2 = 2 * a.T;
  if (tid < kStateDim) s_x[tid] = x_lane;
  __syncthreads();   // every thread's smoothing has read Delta
#pragma unroll
  for (int j = 0; j < kOut; ++j) {
    const int o = tid + j * NT;
    if (o < T2) lds[o] = u_new[j];
  }
  __syncthreads();
  // U, u_0 and the plant state are written through to the device's point of coherence:
  // in a multi-step launch the next step's blocks read them right after the step's signal
  for (int o = tid; o < T2; o += NT) {
    const float v = (o + 2 < T2) ? lds[o + 2] : 0.0f;
    if (writer) store_through(a.Uout + o, v);
    if (u_next) u_next[o] = v;
  }
  if (writer && tid < 2 && u0_out) store_through(u0_out + tid, lds[tid]);
  if (tid >= 64) return;
  const int lane = tid;
  float x[kStateDim];
#pragma unroll
  for (int i = 0; i < kStateDim; ++i) x[i] = s_x[i];
  const float vc0 = fminf(fmaxf(lds[0], a.u_lo0), a.u_hi0);
  const float vc1 = fminf(fmaxf(lds[1], a.u_lo1), a.u_hi1);
  const float in[6] = {x[3], x[4], x[5], x[6], vc0, vc1};
  const bool net = kMayNet && (!kMayBasis || a.model != kModelBasis);
  float f = 0.0f;   // output `lane` of the dynamics (lanes < 4)
  if constexpr (kMayBasis) {
    if (!net && lane < 4) f = basis_out(params, in, vc0, vc1, lane);
  }
  if constexpr (kMayNet) {
    if (net) {
      const int H = HC > 0 ? HC : a.hidden;
      const float* W1 = params;
      const float* b1 = W1 + H * 6;
      const float* W2 = b1 + H;
      const float* b2 = W2 + H * H;
      const float* W3 = b2 + H;
      const float* b3 = W3 + 4 * H;
      const int n = lane < H ? lane : 0;   // the lane's neuron (lanes past H repeat neuron 0)
      const int o = lane & 3;
      if constexpr (PL) {
        static_assert(HC > 0 && HC % 4 == 0, "the plant layout needs a fixed width, a multiple of 4");
        // the same sums in the same order; every weight is read before the first sum
        float4 w2[HC / 4], w3[HC / 4];
#pragma unroll
        for (int q = 0; q < HC / 4; ++q) {
          w2[q] = *reinterpret_cast<const float4*>(W2 + ((q * HC + n) << 2));
          w3[q] = *reinterpret_cast<const float4*>(W3 + ((q * 4 + o) << 2));
        }
        float acc = b1[n];
#pragma unroll
        for (int j = 0; j < 6; ++j) acc = __builtin_fmaf(W1[n * 6 + j], in[j], acc);
        const float h1 = tanh_f(acc);
        acc = b2[n];
#pragma unroll
        for (int q = 0; q < HC / 4; ++q) {
          acc = __builtin_fmaf(w2[q].x, lane_value(h1, 4 * q + 0), acc);
          acc = __builtin_fmaf(w2[q].y, lane_value(h1, 4 * q + 1), acc);
          acc = __builtin_fmaf(w2[q].z, lane_value(h1, 4 * q + 2), acc);
          acc = __builtin_fmaf(w2[q].w, lane_value(h1, 4 * q + 3), acc);
        }
        const float h2 = tanh_f(acc);
        acc = b3[o];
#pragma unroll
        for (int q = 0; q < HC / 4; ++q) {
          acc = __builtin_fmaf(w3[q].x, lane_value(h2, 4 * q + 0), acc);
          acc = __builtin_fmaf(w3[q].y, lane_value(h2, 4 * q + 1), acc);
          acc = __builtin_fmaf(w3[q].z, lane_value(h2, 4 * q + 2), acc);
          acc = __builtin_fmaf(w3[q].w, lane_value(h2, 4 * q + 3), acc);
        }
        f = acc;
      } else {
        float acc = b1[n];
#pragma unroll
        for (int j = 0; j < 6; ++j) acc = __builtin_fmaf(W1[n * 6 + j], in[j], acc);
        const float h1 = tanh_f(acc);
        acc = b2[n];
        if constexpr (HC > 0) {
#pragma unroll
          for (int j = 0; j < HC; ++j) acc = __builtin_fmaf(W2[n * HC + j], lane_value(h1, j), acc);
        } else {
          for (int j = 0; j < H; ++j) acc = __builtin_fmaf(W2[n * H + j], lane_value(h1, j), acc);
        }
        const float h2 = tanh_f(acc);
        acc = b3[o];
        if constexpr (HC > 0) {
#pragma unroll
          for (int j = 0; j < HC; ++j) acc = __builtin_fmaf(W3[o * HC + j], lane_value(h2, j), acc);
        } else {
          for (int j = 0; j < H; ++j) acc = __builtin_fmaf(W3[o * H + j], lane_value(h2, j), acc);
        }
        f = acc;
      }
    }
  }
  const float fo[4] = {lane_value(f, 0), lane_value(f, 1), lane_value(f, 2), lane_value(f, 3)};
  float sth, cth;
  sincosf(x[2], &sth, &cth);
  float y[kStateDim];
  y[0] = x[0] + a.dt * (cth * x[4] - sth * x[5]);
  y[1] = x[1] + a.dt * (sth * x[4] + cth * x[5]);
  y[2] = x[2] + a.dt * x[6];
#pragma unroll
  for (int i = 0; i < 4; ++i) y[3 + i] = x[3 + i] + a.dt * fo[i];
  // component `lane` by lane (lanes < 7), selected with constant indices
  float yl = y[0];
#pragma unroll
  for (int i = 1; i < kStateDim; ++i) yl = lane == i ? y[i] : yl;
  if (lane < kStateDim) {
    if (writer) {
      store_through(const_cast<float*>(a.x0_dev) + lane, yl);
      if (x_copy) store_through(x_copy + lane, yl);
    }
    if (x_next) x_next[lane] = yl;
  }
}

// The final stage of an iteration, run by the one block that merges: the old controls,
// the Savitzky-Golay taps and (receding step) the plant state are loaded early
// (prefetch), so that these loads share a memory round trip with a merge's own;
// apply() then forms Delta = lds[0..2T) * scale,
// smooths it, updates U, writes the statistics and the status, advances the iteration
// counter and, in a receding step, shifts U and advances the plant.
// RECEDE = false: a kernel that never runs a receding step (compiled out).  HC, PL: see
// receding_step.
template <int NT, int MODEL = kModelNet, bool RECEDE = true, int HC = 0, bool PL = false>
struct FinalStage {
  static constexpr int kOut = (2 * kTMax + NT - 1) / NT;
  static constexpr int kTapReg = 16;
  float u_old[kOut];
  float taps[kOut][kTapReg];
  float x_old = 0.0f;   // component tid of the plant state (receding step, threads tid < 7)

  __device__ __forceinline__ void prefetch(const RolloutArgs& a) {
    const int tid = threadIdx.x, T2 = 2 * a.T, w = a.sg_window;
    if constexpr (RECEDE) {
      // one component per thread: vector loads, which unlike a uniform (scalar) load do
      // not hold up the LDS waits of the merge that follows
      x_old = (a.recede && tid < kStateDim) ? load_through(a.x0_dev + tid) : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kOut; ++j) {
      const int o = tid + j * NT;
      u_old[j] = (o < T2) ? load_through(a.Uout + o) : 0.0f;
#pragma unroll
      for (int i = 0; i < kTapReg; ++i)
        taps[j][i] = (o < T2 && w > 1 && w <= kTapReg && i < w) ? a.sg[(size_t)(o >> 1) * w + i] : 0.0f;
    }
  }

  // The same inputs for a block that already holds them: U in LDS (u_lds[2T]) and the
  // plant state in registers (x[7], the same in every thread).
  __device__ __forceinline__ void prefetch_local(const RolloutArgs& a, const float* u_lds, const float (&x)[kStateDim]) {
    const int tid = threadIdx.x, T2 = 2 * a.T, w = a.sg_window;
    if constexpr (RECEDE) {
      x_old = x[0];
#pragma unroll
      for (int i = 1; i < kStateDim; ++i) x_old = tid == i ? x[i] : x_old;
    }
#pragma unroll
    for (int j = 0; j < kOut; ++j) {
      const int o = tid + j * NT;
      u_old[j] = (o < T2) ? u_lds[o] : 0.0f;
#pragma unroll
      for (int i = 0; i < kTapReg; ++i)
        taps[j][i] = (o < T2 && w > 1 && w <= kTapReg && i < w) ? a.sg[(size_t)(o >> 1) * w + i] : 0.0f;
    }
  }

  // iter: the counter word of this iteration (the device counter becomes iter + 1);
  // u0_out, x_copy: the receding step's outputs (nullable).  writer, u_next, x_next: see
  // receding_step (writer = false also leaves the statistics, the status and the counter).
  __device__ __forceinline__ void apply(const RolloutArgs& a, float* lds, bool fin, float scale, const float* params,
                                        float stat0, float stat1, uint32_t iter, float* u0_out, float* x_copy,
                                        bool writer = true, float* u_next = nullptr, float* x_next = nullptr) {
    const int tid = threadIdx.x, T2 = 2 * a.T, w = a.sg_window;
#pragma unroll
    for (int j = 0; j < kOut; ++j) {
      const int o = tid + j * NT;
      if (o < T2) {
        const float d = lds[o] * scale;
        lds[o] = d;
        if (writer) a.stats[2 + o] = d;
      }
    }
    __syncthreads();
    float u_new[kOut];
#pragma unroll
    for (int j = 0; j < kOut; ++j) {
      const int o = tid + j * NT;
      u_new[j] = u_old[j];
      if (o < T2 && fin && a.update_U) {
        float upd;
        if (w == 1) {
          upd = lds[o];
        } else {
          const int t = o >> 1, c = o & 1;
          const int lo = min(max(t - w / 2, 0), a.T - w);
          upd = 0.0f;
          if (w <= kTapReg) {
#pragma unroll
            for (int i = 0; i < kTapReg; ++i)
              if (i < w) upd = __builtin_fmaf(taps[j][i], lds[2 * (lo + i) + c], upd);
          } else {
            const float* row = a.sg + (size_t)t * w;
            for (int i = 0; i < w; ++i) upd = __builtin_fmaf(row[i], lds[2 * (lo + i) + c], upd);
          }
        }
        u_new[j] = u_old[j] + upd;
        if (writer && !a.recede) store_through(a.Uout + o, u_new[j]);
      }
    }
    if (writer && tid == 0) {
      *a.status = fin ? 0 : kStatusNonfinite;
      a.stats[0] = stat0;
      a.stats[1] = stat1;
      if (a.iter_dev) *a.iter_dev = iter + 1u;
    }
    if constexpr (RECEDE) {
      if (a.recede)
        receding_step<NT, kOut, MODEL, HC, PL>(a, u_new, x_old, lds, params, u0_out, x_copy, writer, u_next, x_next);
    }
  }

  // K-shard form: the merged row (rho, eta, N[2T] in lds) of this launch's samples goes to
  // a.row_out in place of the update; U and the statistics are left unchanged.  Called
  // by the whole block.
  __device__ __forceinline__ void export_row(const RolloutArgs& a, const float* lds, float rho, float eta,
                                             uint32_t iter) {
    const int tid = threadIdx.x, T2 = 2 * a.T;
    __syncthreads();
    for (int o = tid; o < T2; o += NT) a.row_out[2 + o] = lds[o];
    if (tid == 0) {
      a.row_out[0] = rho;
      a.row_out[1] = eta;
      *a.status = 0;
      if (a.iter_dev) *a.iter_dev = iter + 1u;
    }
  }
};

// What the final stage of one iteration writes besides U: the counter word of the
// iteration (the device counter becomes iter + 1) and, in a receding step, where u_0 and
// the new plant state are copied (nullable).  A launch that runs several receding steps
// passes each step's own.
struct StepTarget {
  uint32_t iter;
  float* u0_out;
  float* x_copy;
};

// Called by every rollout block with its partial row (rho_g, eta_g and N_g[2T] in
// LDS; tile = the block's index among the launch's blocks of this problem).  Blocks
// arrive in groups of merge_group_size(G); the last to arrive in a group merges the
// group's rows, and the last group merger merges the group rows and applies
// Algorithm 2's normalisation, the Savitzky-Golay smoothing and the update
// U <- U + SG * Delta.  With a single group the second level is skipped (merging one
// row with scale exp(0) = 1 would return it unchanged).  Every decision is uniform
// over the block, so all barriers are reached by all threads.  Returns, in every
// thread, whether this block ran the final stage.
template <int NT, int MODEL = kModelNet, bool RECEDE = true, int HC = 0>
__device__ bool finish_iteration(const RolloutArgs& a, int tile, float rho_b, float eta_b,
                                 const float* N_lds /* [2T] */, float* lds /* >= 2T floats */,
                                 const float* params = nullptr /* the model's parameters in LDS, or a.params */,
                                 const StepTarget* target = nullptr /* default: a.nk.iter, a.u0_out, a.x_copy */) {
  if (!params) params = a.params;
  const StepTarget st = target ? *target : StepTarget{a.nk.iter, a.u0_out, a.x_copy};
  bool ran_final = false;
  __shared__ unsigned s_flag;
  __shared__ float s_small[2 * kMergeChunk];
  const int tid = threadIdx.x;
  const int T2 = 2 * a.T;
  const int stride = 2 + T2;
  const int gsz = merge_group_size(a.G);
  const int ngrp = (a.G + gsz - 1) / gsz;
  const int grp = tile / gsz;
  const int n_in = min(gsz, a.G - grp * gsz);
  __syncthreads();
  if (publish_and_count<NT>(a.part + (size_t)tile * stride, rho_b, eta_b, N_lds, T2, a.cnt + grp,
                            (unsigned)n_in, &s_flag)) {
    // what the final stage needs (the old controls, the smoothing taps, the plant state)
    // is loaded by every group merger while its group row's count is in flight (or
    // before the merge when there is a single group), so that the final merge finds it
    // in registers
    FinalStage<NT, MODEL, RECEDE, HC> fs;
    float rho, eta;
    bool final_merge = ngrp == 1;
    if (final_merge) fs.prefetch(a);
    merge_rows<NT>(a.part + (size_t)grp * gsz * stride, n_in, stride, T2, a.inv_lambda, lds, s_small,
                   rho, eta);
    if (tid == 0) __hip_atomic_store(a.cnt + grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ngrp > 1) {
      __syncthreads();
      final_merge = publish_and_count<NT>(a.part2 + (size_t)grp * stride, rho, eta, lds, T2, a.cnt + ngrp,
                                          (unsigned)ngrp, &s_flag, [&] { fs.prefetch(a); });
      if (final_merge) {
        merge_rows<NT>(a.part2, ngrp, stride, T2, a.inv_lambda, lds, s_small, rho, eta);
        if (tid == 0) __hip_atomic_store(a.cnt + ngrp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (final_merge) {
      ran_final = true;
      if (a.row_out) {
        fs.export_row(a, lds, rho, eta, st.iter);
      } else {
        const bool fin = (rho < kInf) && (eta > 0.0f);
        fs.apply(a, lds, fin, fin ? 1.0f / eta : 0.0f, params, rho, fin ? eta : 0.0f, st.iter, st.u0_out,
                 st.x_copy);
      }
    }
  }
  __syncthreads();
  return ran_final;
}

}  // namespace mppi
