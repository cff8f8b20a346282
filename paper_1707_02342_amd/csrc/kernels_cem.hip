// Algorithm 3 (cross-entropy weights): the update that follows a rollout launch run
// with cem_zeta > 0.  That launch leaves every sample's cost S[k] and its delta row
// D[k][T][2] (delta = v - u) in global memory; this single block of 1024 threads
//   1. counts the finite costs n and takes zeta' = min(zeta, n),
//   2. finds the elite threshold -- the zeta'-th smallest cost -- by a radix select on
//      order-preserving integer keys, starting below the bits that the smallest and the
//      largest finite key share, so that the first digit already spreads the keys,
//   3. lists the elite samples in sample order (equal costs at the threshold go to the
//      lower sample index), and sums their delta rows with compensated additions,
//   4. applies U <- U + SGF * (sum / zeta') and, in a receding step, the shift and the
//      plant step (the same final stage as Algorithm 2's merge).
// With several blocks (gridDim.x > 1) every block takes steps 1-3 in full except that it
// sums only its share of the elite rows (global wave w of the launch takes list entries
// w, w + W, ...); the blocks publish their partial sums as Algorithm 2's merge publishes
// its rows, and the last to arrive adds them in block order and takes step 4.  One CU
// alone cannot pull the elite rows quickly (about 307 KB at K = 1920).
// The costs stay in registers when K <= 8192 (one memory round trip); larger K is
// processed in chunks of 8192 samples.
#include "kernels_common.hip.h"

namespace mppi {

constexpr int kCemBlock = 1024;
constexpr int kCemWaves = kCemBlock / 64;
constexpr int kCemKeys = 8;                       // keys per thread and chunk
constexpr int kCemChunk = kCemBlock * kCemKeys;   // samples per chunk

// Monotone map of a cost to an unsigned key (-0 and +0 alike); the cost of a non-finite
// sample (+inf) maps above every finite cost, and padding (0xFFFFFFFF) above that.
__device__ __forceinline__ unsigned cost_key(float s) {
  const unsigned b = __float_as_uint(s + 0.0f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_cost(unsigned key) {
  return __uint_as_float((key & 0x80000000u) ? (key & 0x7FFFFFFFu) : ~key);
}
constexpr unsigned kInfKey = 0xFF800000u;   // cost_key(+inf)
constexpr unsigned kPadKey = 0xFFFFFFFFu;

// Exclusive prefix sum of v over the block in thread order; total = the block's sum.
__device__ __forceinline__ int cem_excl_sum(int v, int* s_w, int& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int n = __shfl_up(incl, d, 64);
    if (lane >= d) incl += n;
  }
  if (lane == 63) s_w[wv] = incl;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kCemWaves; ++i) {
    const int c = s_w[i];
    base += (i < wv) ? c : 0;
    tot += c;
  }
  __syncthreads();
  total = tot;
  return base + incl - v;
}

// NCOL: float2 columns per lane, 2 for T <= 128, 4 for T <= 256.  HC: the network width
// when the context's network is 32 wide (unrolled plant step), else 0.
template <int NCOL, int HC>
__global__ __launch_bounds__(kCemBlock) void cem_update_kernel(RolloutArgs a) {
  if (a.iter_dev) a.nk.iter = *a.iter_dev;   // advanced by the final stage
  constexpr int kBatch = NCOL == 2 ? 12 : 4;   // rows per wave whose loads are in flight together
  __shared__ unsigned s_hist[256];
  __shared__ int s_w[kCemWaves];
  __shared__ unsigned s_red[3 * kCemWaves];
  __shared__ unsigned s_sel[4];
  __shared__ unsigned s_cand[64];
  __shared__ int s_list[kCemChunk];
  __shared__ float s_part[kCemWaves][2 * kTMax];
  __shared__ float s_delta[2 * kTMax];
  __shared__ unsigned s_flag;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K = a.K, T2 = 2 * a.T;
  const int nchunk = (K + kCemChunk - 1) / kCemChunk;
  const bool resident = nchunk == 1;

  FinalStage<kCemBlock, kModelAny, true, HC> fs;
  fs.prefetch(a);

  unsigned key[kCemKeys];
  auto load_keys = [&](int c0) {
#pragma unroll
    for (int i = 0; i < kCemKeys; ++i) {
      const int k = c0 + tid * kCemKeys + i;
      key[i] = (k < K) ? cost_key(a.S[k]) : kPadKey;
    }
  };

  // 1. finite count and the smallest / largest finite key
  unsigned nf = 0u, kmin = kPadKey, kmax = 0u;
  for (int c = 0; c < nchunk; ++c) {
    load_keys(c * kCemChunk);
#pragma unroll
    for (int i = 0; i < kCemKeys; ++i) {
      if (key[i] < kInfKey) {
        ++nf;
        kmin = min(kmin, key[i]);
        kmax = max(kmax, key[i]);
      }
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    nf += __shfl_xor(nf, m, 64);
    kmin = min(kmin, (unsigned)__shfl_xor(kmin, m, 64));
    kmax = max(kmax, (unsigned)__shfl_xor(kmax, m, 64));
  }
  if (lane == 0) {
    s_red[wv] = nf;
    s_red[kCemWaves + wv] = kmin;
    s_red[2 * kCemWaves + wv] = kmax;
  }
  __syncthreads();
  nf = 0u;
  kmin = kPadKey;
  kmax = 0u;
#pragma unroll
  for (int i = 0; i < kCemWaves; ++i) {
    nf += s_red[i];
    kmin = min(kmin, s_red[kCemWaves + i]);
    kmax = max(kmax, s_red[2 * kCemWaves + i]);
  }
  const int zeff = min(a.cem_zeta, (int)nf);

  // 2. radix select of the zeff-th smallest key
  unsigned zkey = kInfKey;
  int need_eq = 0;
  unsigned eq_total = 0u;   // keys equal to the threshold key
  if (zeff > 0) {
    const unsigned diff = kmin ^ kmax;
    int nb = diff ? 32 - __clz(diff) : 0;            // bits below the shared prefix
    unsigned mask = nb == 32 ? 0u : ~((1u << nb) - 1u);
    unsigned prefix = kmin & mask;
    unsigned r = (unsigned)zeff;
    while (nb > 0) {
      const int width = min(8, nb);
      const int shift = nb - width;
      const unsigned dmask = (1u << width) - 1u;
      for (int i = tid; i < 256; i += kCemBlock) s_hist[i] = 0u;
      __syncthreads();
      for (int c = 0; c < nchunk; ++c) {
        if (!resident) load_keys(c * kCemChunk);
#pragma unroll
        for (int i = 0; i < kCemKeys; ++i)
          if ((key[i] & mask) == prefix) atomicAdd(&s_hist[(key[i] >> shift) & dmask], 1u);
      }
      __syncthreads();
      if (tid < 64) {
        const unsigned c0 = s_hist[4 * tid], c1 = s_hist[4 * tid + 1];
        const unsigned c2 = s_hist[4 * tid + 2], c3 = s_hist[4 * tid + 3];
        const unsigned own = c0 + c1 + c2 + c3;
        unsigned incl = own;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const unsigned n = __shfl_up(incl, d, 64);
          if (tid >= d) incl += n;
        }
        unsigned before = incl - own;
        if (before < r && r <= incl) {
          unsigned b = 4u * tid;
          if (r > before + c0) {
            before += c0;
            ++b;
            if (r > before + c1) {
              before += c1;
              ++b;
              if (r > before + c2) {
                before += c2;
                ++b;
              }
            }
          }
          s_sel[0] = b;
          s_sel[1] = r - before;
          s_sel[2] = b == 4u * tid ? c0 : (b == 4u * tid + 1u ? c1 : (b == 4u * tid + 2u ? c2 : c3));
          s_sel[3] = 0u;
        }
      }
      __syncthreads();
      prefix |= s_sel[0] << shift;
      mask |= dmask << shift;
      r = s_sel[1];
      nb = shift;
      if (nb > 0 && s_sel[2] <= 64u) {
        // few keys left in the selected bin: rank them directly instead of more passes
        for (int c = 0; c < nchunk; ++c) {
          if (!resident) load_keys(c * kCemChunk);
#pragma unroll
          for (int i = 0; i < kCemKeys; ++i)
            if ((key[i] & mask) == prefix) s_cand[atomicAdd(&s_sel[3], 1u)] = key[i];
        }
        __syncthreads();
        if (tid < 64) {
          const unsigned n = s_sel[3];
          const unsigned my = tid < (int)n ? s_cand[tid] : kPadKey;
          unsigned lt = 0u, le = 0u;
          for (unsigned j = 0; j < n; ++j) {
            const unsigned c = s_cand[j];
            lt += c < my ? 1u : 0u;
            le += c <= my ? 1u : 0u;
          }
          // every lane holding the selected key writes the same two values
          if (tid < (int)n && lt < r && r <= le) {
            s_sel[0] = my;
            s_sel[1] = r - lt;
            s_sel[2] = le - lt;
          }
        }
        __syncthreads();
        prefix = s_sel[0];
        r = s_sel[1];
        nb = 0;
      }
    }
    zkey = prefix;
    need_eq = (int)r;
    // the last pass (or the direct ranking) left the count of keys equal to zkey in s_sel[2];
    // when the first pass already isolated one key value (nb = 0 from the start) count them
    eq_total = diff ? s_sel[2] : nf;
  }

  // 3. elite rows, summed in list order per wave (compensated), chunk by chunk
  Acc acc[NCOL][2];
#pragma unroll
  for (int j = 0; j < NCOL; ++j) acc[j][0] = acc[j][1] = Acc{0.0f, 0.0f};
  if (zeff > 0) {
    int eq_taken = 0;
    for (int c = 0; c < nchunk; ++c) {
      const int c0 = c * kCemChunk;
      if (!resident) load_keys(c0);
      int n_eq = 0;
#pragma unroll
      for (int i = 0; i < kCemKeys; ++i) n_eq += key[i] == zkey ? 1 : 0;
      int tot_eq = 0, tot_el;
      // when every key equal to the threshold is elite, no ranking among them is needed
      int eq_rank = 0;
      if (need_eq >= (int)eq_total) tot_eq = 0;
      else eq_rank = eq_taken + cem_excl_sum(n_eq, s_w, tot_eq);
      const bool all_eq = need_eq >= (int)eq_total;
      int n_el = 0;
      unsigned take = 0u;
#pragma unroll
      for (int i = 0; i < kCemKeys; ++i) {
        bool el = key[i] < zkey;
        if (key[i] == zkey) {
          el = all_eq || eq_rank < need_eq;
          ++eq_rank;
        }
        take |= el ? (1u << i) : 0u;
        n_el += el ? 1 : 0;
      }
      int pos = cem_excl_sum(n_el, s_w, tot_el);
#pragma unroll
      for (int i = 0; i < kCemKeys; ++i)
        if (take & (1u << i)) s_list[pos++] = c0 + tid * kCemKeys + i;
      eq_taken += tot_eq;
      __syncthreads();
      // global wave gw sums list entries gw, gw + W, ...; lane owns float2 columns lane + 64 j
      const int gw = blockIdx.x * kCemWaves + wv, W = gridDim.x * kCemWaves;
      for (int e0 = gw; e0 < tot_el; e0 += W * kBatch) {
        float2 v[kBatch][NCOL];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const int e = e0 + b * W;
          const float2* row = reinterpret_cast<const float2*>(a.D + (size_t)s_list[min(e, tot_el - 1)] * T2);
#pragma unroll
          for (int j = 0; j < NCOL; ++j) {
            const int col = lane + 64 * j;
            v[b][j] = (e < tot_el && 2 * col < T2) ? row[col] : make_float2(0.0f, 0.0f);
          }
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          if (e0 + b * W < tot_el) {
#pragma unroll
            for (int j = 0; j < NCOL; ++j) {
              acc[j][0].add(v[b][j].x);
              acc[j][1].add(v[b][j].y);
            }
          }
        }
      }
      __syncthreads();
    }
  }
  // 4. the waves' partial sums in wave order, then the final stage
#pragma unroll
  for (int j = 0; j < NCOL; ++j) {
    const int col = lane + 64 * j;
    if (2 * col < T2) {
      s_part[wv][2 * col] = acc[j][0].value();
      s_part[wv][2 * col + 1] = acc[j][1].value();
    }
  }
  __syncthreads();
  if (tid < T2) {
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < kCemWaves; ++w) s += s_part[w][tid];
    s_delta[tid] = s;
  }
  if (gridDim.x > 1) {
    // the block's share, published like a rollout block's row (a.part, a.cnt[0]: unused
    // by a rollout launch that stores delta rows); the last block adds the shares
    const int stride = 2 + T2;
    __syncthreads();
    if (!publish_and_count<kCemBlock>(a.part + (size_t)blockIdx.x * stride, 0.0f, 0.0f, s_delta, T2, a.cnt,
                                      gridDim.x, &s_flag))
      return;
    if (tid == 0) a.cnt[0] = 0u;
    if (tid < T2) {
      float s = 0.0f;
      for (int b = 0; b < (int)gridDim.x; ++b) s += load_through(a.part + (size_t)b * stride + 2 + tid);
      s_delta[tid] = s;
    }
  }
  fs.apply(a, s_delta, zeff > 0, zeff > 0 ? 1.0f / (float)zeff : 0.0f, a.params, key_cost(zkey), (float)zeff,
           a.nk.iter, a.u0_out, a.x_copy);
}

template __global__ void cem_update_kernel<2, 0>(RolloutArgs);
template __global__ void cem_update_kernel<4, 0>(RolloutArgs);
template __global__ void cem_update_kernel<2, 32>(RolloutArgs);
template __global__ void cem_update_kernel<4, 32>(RolloutArgs);

}  // namespace mppi
