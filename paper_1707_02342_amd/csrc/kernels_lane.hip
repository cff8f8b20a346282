// Rollout schedule "lane": one wavefront lane per sample.
//
// Every lane carries its sample's full state through the T-step loop in
// registers (Algorithm 1's inner loop), drawing eps from Philox on the fly, and
// evaluates the dynamics network through a policy:
//
//  * NetUniform<H> (FP32): each lane runs its own network; the weights are read with
//    wave-uniform addresses, so the compiler serves them from the scalar cache as
//    SGPR operands.
//  * NetMfma<P, H> (BF16 or FP16 operands, FP32 accumulation): the wave's 64 samples
//    form four 16-sample columns of one batched product per layer on the matrix
//    cores, out^T = W in^T (neurons x samples), with v_mfma_f32_16x16x32_{bf16,f16}.
//    Its accumulator layout (lane = column + 16 * (row / 4), four rows per lane) is
//    turned into the next layer's operand layout (lane = column + 16 * (k / 8), eight
//    k per lane) without moving data between lanes, by ordering the weight matrix's
//    k-dimension to match what each lane already holds.  Layer 3's rows are placed so
//    that every lane receives the four outputs of its own sample.
//
//  * NetBasis (FP32): the basis-function model, f = Theta^T phi(x_d, v).
//
// Cost, weights and the update stay FP32 in all.  This is the throughput schedule
// for large K: one sample per lane keeps every lane busy.
#include "kernels_common.hip.h"

namespace mppi {

constexpr int kLaneBlock = 256;
constexpr int kLaneWaves = kLaneBlock / 64;

// ---------------------------------------------------------------------------
// FP32 network, one per lane
// ---------------------------------------------------------------------------
template <int HID>
struct NetUniform {
  static constexpr int kModel = kModelNet;
  static constexpr int kHidden = HID;
  const float* __restrict__ P;
  __device__ explicit NetUniform(const float* p) : P(p) {}
  __device__ __forceinline__ void eval(const float in[6], float f[4]) const {
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
};

// ---------------------------------------------------------------------------
// Basis-function model, one per lane (Theta read with wave-uniform addresses)
// ---------------------------------------------------------------------------
struct NetBasis {
  static constexpr int kModel = kModelBasis;
  static constexpr int kHidden = 0;
  const float* __restrict__ P;
  __device__ explicit NetBasis(const float* p) : P(p) {}
  __device__ __forceinline__ void eval(const float in[6], float f[4]) const { basis_f(P, in, in[4], in[5], f); }
};

// ---------------------------------------------------------------------------
// BF16 / FP16 network on the matrix cores, one wave = 64 samples
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

constexpr int kPrecBF16 = 1;
constexpr int kPrecFP16 = 2;

template <int PREC> struct MfmaOps;
template <> struct MfmaOps<kPrecBF16> {
  typedef bf16x8 vec;
  static __device__ __forceinline__ f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ vec pack(const float v[8]) {
    vec r;
#pragma unroll
    for (int c = 0; c < 8; ++c) r[c] = (__bf16)v[c];
    return r;
  }
};
template <> struct MfmaOps<kPrecFP16> {
  typedef f16x8 vec;
  static __device__ __forceinline__ f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ vec pack(const float v[8]) {
    vec r;
#pragma unroll
    for (int c = 0; c < 8; ++c) r[c] = (_Float16)v[c];
    return r;
  }
};

// Neuron held in k-slot c of lane group g for k-block kb: exactly what a lane holds
// of the previous layer's accumulators (neurons 16 m + 4 g + r, m = 2 kb + c / 4,
// r = c % 4), so the activations never leave their lane.
__device__ __forceinline__ int kslot_neuron(int kb, int g, int c) {
  return 16 * (2 * kb + (c >> 2)) + 4 * g + (c & 3);
}

template <int PREC, int HID>
struct NetMfma {
  static constexpr int kModel = kModelNet;
  static constexpr int kHidden = HID;
  typedef MfmaOps<PREC> Ops;
  typedef typename Ops::vec vec;
  static constexpr int NM = HID / 16;   // 16-neuron tiles
  static constexpr int NKB = HID / 32;  // 32-wide k-blocks of layers 2 and 3
  vec A1[NM];             // [W1 row | b1 | 0] per tile, the same in every lane group
  vec A2[NM][NKB];
  vec A3[4][NKB];         // rows 4q..4q+3 hold W3 for the samples of column block q
  f32x4 C2[NM];           // b2 in accumulator layout
  f32x4 C3;               // b3 in accumulator layout
  int g;                  // lane group (lane / 16)

  __device__ explicit NetMfma(const float* __restrict__ P) {
    const float* W1 = P;
    const float* b1 = W1 + HID * 6;
    const float* W2 = b1 + HID;
    const float* b2 = W2 + HID * HID;
    const float* W3 = b2 + HID;
    const float* b3 = W3 + 4 * HID;
    const int lane = threadIdx.x & 63;
    g = lane >> 4;
    const int i = lane & 15;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      float v[8];
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] = W1[(16 * m + i) * 6 + c];
      v[6] = b1[16 * m + i];
      v[7] = 0.0f;
      A1[m] = Ops::pack(v);
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = W2[(16 * m + i) * HID + kslot_neuron(kb, g, c)];
        A2[m][kb] = Ops::pack(v);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) C2[m][r] = b2[16 * m + 4 * g + r];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        float v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = (i >> 2) == q ? W3[(i & 3) * HID + kslot_neuron(kb, g, c)] : 0.0f;
        A3[q][kb] = Ops::pack(v);
      }
#pragma unroll
    for (int r = 0; r < 4; ++r) C3[r] = b3[r];
  }

  // One network evaluation for the wave's 64 samples (every lane must call it).
  // Lane l supplies its own sample's inputs and receives its own sample's outputs.
  __device__ __forceinline__ void eval(const float in[6], float f[4]) const {
    bool fin = true;
#pragma unroll
    for (int c = 0; c < 6; ++c) fin = fin && finite_f(in[c]);
    float v[8];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = fin ? in[c] : 0.0f;   // other columns must stay finite
    v[6] = 1.0f;
    v[7] = 0.0f;
    const u32x4 b1u = __builtin_bit_cast(u32x4, Ops::pack(v));
    const u32x4 zero = {0u, 0u, 0u, 0u};
    // layer 1: column block q reads only the operand slots of lane group q
    f32x4 D1[NM][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const vec bq = __builtin_bit_cast(vec, g == q ? b1u : zero);
#pragma unroll
      for (int m = 0; m < NM; ++m) D1[m][q] = Ops::mma(A1[m], bq, f32x4{0.0f, 0.0f, 0.0f, 0.0f});
    }
    // layer 2
    f32x4 D2[NM][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      vec B2[NKB];
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        float h[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) h[c] = tanh_f(D1[2 * kb + (c >> 2)][q][c & 3]);
        B2[kb] = Ops::pack(h);
      }
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        f32x4 acc = C2[m];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) acc = Ops::mma(A2[m][kb], B2[kb], acc);
        D2[m][q] = acc;
      }
    }
    // layer 3: outputs of column block q land in rows 4q..4q+3, i.e. in lane group q
    f32x4 D3 = C3;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        float h[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) h[c] = tanh_f(D2[2 * kb + (c >> 2)][q][c & 3]);
        D3 = Ops::mma(A3[q][kb], Ops::pack(h), D3);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) f[r] = D3[r];
  }
};

// ---------------------------------------------------------------------------
// Block partial and kernel
// ---------------------------------------------------------------------------

// This block's (rho_g, eta_g, N_g[T][2]), N_g regenerating eps; N_g goes to N_lds
// (complete after the block's next barrier).
// delta_{k,t} = v_{k,t} - u_t (eps, or eps - u_t for exploration samples) in place of
// eps; sU is the nominal sequence in LDS and may alias N_lds.
__device__ __forceinline__ void lane_block_partial(const RolloutArgs& a, float S, bool valid, int k,
                                                   float* red /* [kLaneWaves][2*kTMax] */,
                                                   float* scratch, const float* sU, float* N_lds,
                                                   float& rho_out, float& eta_out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const float sv = valid ? S : kInf;
  const float rho = block_min<kLaneWaves>(sv, scratch);
  const float e = rel_weight(sv, rho, a.inv_lambda);
  const float eta = block_sum<kLaneWaves>(e, scratch);
  for (int t = 0; t < a.T; ++t) {
    float e0 = 0.0f, e1 = 0.0f;
    if (valid) {
      draw_eps((uint32_t)t, (uint32_t)k, a.nk, e0, e1);
      if (k >= a.K_imp) {
        e0 -= sU[2 * t];
        e1 -= sU[2 * t + 1];
      }
    }
    const float n0 = wave_sum(e * e0);
    const float n1 = wave_sum(e * e1);
    if (lane == 0) {
      red[w * 2 * kTMax + 2 * t] = n0;
      red[w * 2 * kTMax + 2 * t + 1] = n1;
    }
  }
  __syncthreads();
  for (int o = threadIdx.x; o < 2 * a.T; o += kLaneBlock) {
    float s = red[o];
#pragma unroll
    for (int i = 1; i < kLaneWaves; ++i) s += red[i * 2 * kTMax + o];
    N_lds[o] = s;
  }
  rho_out = rho;
  eta_out = eta;
}

// One tile of 256 samples of one problem (samples tile*256 ... tile*256 + 255).
template <class Net, bool RECEDE = true>
__device__ void lane_rollout_tile(const RolloutArgs& a, int tile, float* sU, float* red, float* scratch) {
  for (int i = threadIdx.x; i < 2 * a.T; i += kLaneBlock) sU[i] = a.U[i];
  __syncthreads();
  const int k = tile * kLaneBlock + threadIdx.x;
  const bool valid = k < a.K;
  const bool zm = k >= a.K_imp;   // exploration sample: v = eps
  const Net net(a.params);
  // State and cost in compensated form (hi + lo); the network and the kinematics read
  // the hi parts, the cost reads hi + lo.  Lanes past K run too (the matrix-core
  // network needs every lane of the wave) and are discarded.
  Acc x[kStateDim];
#pragma unroll
  for (int i = 0; i < kStateDim; ++i) {
    x[i].hi = a.x0_dev ? a.x0_dev[i] : a.x0[i];
    x[i].lo = 0.0f;
  }
  Acc S{0.0f, 0.0f};
  bool ok = true;
  for (int t = 0; t < a.T; ++t) {
    float e0, e1;
    draw_eps((uint32_t)t, (uint32_t)k, a.nk, e0, e1);
    const float u0 = sU[2 * t], u1 = sU[2 * t + 1];
    const float vc0 = fminf(fmaxf(zm ? e0 : u0 + e0, a.u_lo0), a.u_hi0);
    const float vc1 = fminf(fmaxf(zm ? e1 : u1 + e1, a.u_lo1), a.u_hi1);
    const float d0 = zm ? e0 - u0 : e0, d1 = zm ? e1 - u1 : e1;   // v - u
    const float in[6] = {x[3].hi, x[4].hi, x[5].hi, x[6].hi, vc0, vc1};
    float f[4];
    net.eval(in, f);
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
    S.add(a.gcs0 * (u0 * d0) + a.gcs1 * (u1 * d1));
  }
  float Sv = S.value();
  if (!ok || !finite_f(Sv)) Sv = kInf;
  if (valid) store_through(a.S + k, Sv);   // read by the host or Algorithm 3's update
  if (a.cem_zeta > 0) {
    // Algorithm 3: the sample's delta row, for the elite average
    if (valid) {
      float* drow = a.D + (size_t)k * 2 * a.T;
      for (int t = 0; t < a.T; ++t) {
        float e0, e1;
        draw_eps((uint32_t)t, (uint32_t)k, a.nk, e0, e1);
        if (zm) {
          e0 -= sU[2 * t];
          e1 -= sU[2 * t + 1];
        }
        drow[2 * t] = e0;
        drow[2 * t + 1] = e1;
      }
    }
    return;   // the cross-entropy update runs in the launch that follows
  }
  float rho, eta;
  lane_block_partial(a, Sv, valid, k, red, scratch, sU, sU, rho, eta);
  finish_iteration<kLaneBlock, Net::kModel, RECEDE, Net::kHidden>(a, tile, rho, eta, sU, red);
}

template <class Net>
__global__ __launch_bounds__(kLaneBlock) void rollout_lane_kernel(RolloutArgs a) {
  if (a.iter_dev) a.nk.iter = *a.iter_dev;   // the device counter, advanced by the final merge
  __shared__ float sU[2 * kTMax];
  __shared__ float red[kLaneWaves * 2 * kTMax];
  __shared__ float scratch[kLaneWaves];
  lane_rollout_tile<Net>(a, blockIdx.x, sU, red, scratch);
}

// Batched form: many independent problems (instances) in one persistent launch.
// items[b] = (instance, tile); each block takes items from the launch's work queue in
// the order of the list.  Each instance's noise uses its own iteration counter
// (advanced by its final merge) and its index as the fourth Philox counter word.  A
// tile's work and an instance's merge order do not depend on which block runs it, so
// results are the same for every grid size and item order.
__global__ __launch_bounds__(kLaneBlock) void rollout_batch_kernel(const RolloutArgs* __restrict__ inst,
                                                                 const int2* __restrict__ items,
                                                                 int n_items, const float* __restrict__ map,
                                                                 const float* __restrict__ params,
                                                                 const float* __restrict__ decay,
                                                                 unsigned* __restrict__ queue) {
  __shared__ float sU[2 * kTMax];
  __shared__ float red[kLaneWaves * 2 * kTMax];
  __shared__ float scratch[kLaneWaves];
  for (;;) {
    const int b = next_work_item(queue, n_items);
    if (b < 0) break;
    const int2 it = items[b];
    RolloutArgs a = inst[it.x];
    // the shared inputs come from kernel arguments, so that the weights are read with
    // scalar loads (through pointers loaded from memory they would be generic, loaded
    // per lane and kept in registers)
    a.map = map;
    a.params = params;
    a.decay = decay;
    a.nk.iter = *a.iter_dev;
    lane_rollout_tile<NetUniform<32>, false>(a, it.y, sU, red, scratch);
  }
}

template __global__ void rollout_lane_kernel<NetUniform<32>>(RolloutArgs);
template __global__ void rollout_lane_kernel<NetUniform<64>>(RolloutArgs);
template __global__ void rollout_lane_kernel<NetMfma<kPrecBF16, 32>>(RolloutArgs);
template __global__ void rollout_lane_kernel<NetMfma<kPrecBF16, 64>>(RolloutArgs);
template __global__ void rollout_lane_kernel<NetMfma<kPrecFP16, 32>>(RolloutArgs);
template __global__ void rollout_lane_kernel<NetMfma<kPrecFP16, 64>>(RolloutArgs);

// Launch helper used by the host runtime (keeps the policy types in this file).
hipError_t launch_lane(int precision, int hidden, dim3 grid, hipStream_t stream, const RolloutArgs& a) {
  if (precision == kPrecBF16) {
    if (hidden == 32) rollout_lane_kernel<NetMfma<kPrecBF16, 32>><<<grid, dim3(kLaneBlock), 0, stream>>>(a);
    else rollout_lane_kernel<NetMfma<kPrecBF16, 64>><<<grid, dim3(kLaneBlock), 0, stream>>>(a);
  } else if (precision == kPrecFP16) {
    if (hidden == 32) rollout_lane_kernel<NetMfma<kPrecFP16, 32>><<<grid, dim3(kLaneBlock), 0, stream>>>(a);
    else rollout_lane_kernel<NetMfma<kPrecFP16, 64>><<<grid, dim3(kLaneBlock), 0, stream>>>(a);
  } else if (a.model == kModelBasis) {
    rollout_lane_kernel<NetBasis><<<grid, dim3(kLaneBlock), 0, stream>>>(a);
  } else {
    if (hidden == 32) rollout_lane_kernel<NetUniform<32>><<<grid, dim3(kLaneBlock), 0, stream>>>(a);
    else rollout_lane_kernel<NetUniform<64>><<<grid, dim3(kLaneBlock), 0, stream>>>(a);
  }
  return hipGetLastError();
}

}  // namespace mppi
