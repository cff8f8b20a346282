// Rollout schedule "wave", split form: the 32-lanes-per-sample layout of the wave
// kernel (two samples per wavefront, eight per block) with the block doubled to eight
// waves, so that every SIMD holds a chain wave and a cost wave of the same two samples.
// For the latency-bound regime where a launch fits the device in one block per CU
// (K up to 8 x CUs, e.g. K = 1920) and horizons up to 128 steps.
//
// Only the dynamic states x_d form a serial chain (the network never reads the pose,
// Section VI-B); the noise and the clamp of Algorithm 1 precede it and the kinematics
// and state cost of Section VI-C follow it.  So:
//
//  all waves: draw the noise of every sample and step of the block and form the
//    clamped controls g(v) (network) or the control-only terms (basis model) in LDS;
//  chain wave (waves 0..3, raised issue priority): runs the chain as the wave kernel's
//    deferred form does -- layer 1 from quad_perm DPP operands, layer 2 in row_ror DPP
//    operands of v_fmac_f32 and a v_permlane16_swap, layer 3 (times dt) as a
//    reduce-scatter, the uncompensated state hi_{t+1} = hi_t + y_t and its increment
//    y_t stored to LDS -- and publishes each finished chunk of steps with a
//    workgroup-scope release of a per-pair counter in LDS.  The chunks hold 32 steps
//    except the first, which holds the remainder of T: a chunk costs the cost wave
//    about the same time whatever its length, and with the short chunk first the cost
//    wave has finished every chunk but the last when the chain ends;
//  cost wave (waves 4..7): follows the chain one chunk behind: for chunk c it waits
//    (acquire) for the chain's counter, forms the compensated states x_d(t) = hi_t + lo_t
//    (the two-sum errors of the chain's sums, scanned across the lanes), the heading and
//    the position by compensated scans carried from chunk to chunk, and the state and
//    control costs of the chunk's steps (one step per lane).
//
// The cost wave waits only for the chain of its own block, which never waits, so every
// wait ends.  After both roles, all 512 threads form the block's softmin partial from the
// eight costs and the noise rows, and finish_iteration merges and updates as in every
// rollout kernel.  The costs equal the wave kernel's up to the summation order of the
// compensation terms and of the kinematic scans.
//
// Multi-step receding launch (the MULTI instances with n_steps > 1, launched
// cooperatively so that every block is resident): G rollout blocks and one merger block
// per merge group.  A rollout block loops over the steps, keeping the chain's network
// constants in registers and the model's parameters (for the plant step) in LDS.  At the
// end of step s it writes its row through, waits for those stores, and writes the step
// into its arrival word; it draws step s + 1's noise (which does not depend on U) and
// waits until its copy of the group words shows step s for every group; it then merges
// the group rows and runs the final stage itself -- normalisation, smoothing, update,
// shift, plant step -- so that step s + 1 starts from U and the plant state in its own
// LDS with no further memory round trip.  Every block computes the same values in the
// same order; block 0 alone writes U, the plant state, the statistics and the histories.
// A merger block waits until its group's arrival words show step s, merges the group's
// rows into the group row and writes the step into every copy of its group word.  Every
// signal is a word written through after the data it announces has reached the device's
// point of coherence, and read with device-coherent loads; every word holds a step
// number that only grows, so none is reset.  (Counting arrivals with atomic adds and
// polling the count took ~4.5 us to be seen by the poller, against ~0.6 us for a written
// word.)  Every wait is bounded: a block that gives up sets the status and leaves.  The
// results equal those of one launch per step bit for bit.
#include "wave_common.hip.h"

namespace mppi {

constexpr int kSplitBlock = 512;   // 4 chain waves + 4 cost waves, 8 samples
constexpr int kSplitPairs = 4;     // sample pairs per block (one chain and one cost wave each)
// floats of the model's parameters a multi-step launch stages in LDS (the space is sized
// for the 6-32-32-4 network, 1412 floats; the basis model stages its Theta, 100)
constexpr int kSplitParams = 6 * 32 + 32 + 32 * 32 + 32 + 4 * 32 + 4;
constexpr int kSplitBasisParams = 25 * 4;

// the plant layout moves each of the network's parameters to a place of its own in the
// same space, and its 16-byte words (the W2 and W3 sections) start on 16-byte boundaries
constexpr bool plant_layout_fits() {
  bool seen[kSplitParams] = {};
  for (int i = 0; i < kSplitParams; ++i) {
    const int d = plant_layout_index(i, 32);
    if (d < 0 || d >= kSplitParams || seen[d]) return false;
    seen[d] = true;
  }
  return (7 * 32) % 4 == 0 && (8 * 32 + 32 * 32) % 4 == 0;
}
static_assert(plant_layout_fits(), "the plant layout must permute the 6-32-32-4 parameter vector");

namespace {

__device__ __forceinline__ void wait_count(unsigned* f, unsigned v) {
  while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < v) __builtin_amdgcn_s_sleep(1);
}

__device__ __forceinline__ void publish_count(unsigned* f, unsigned v) {
  __hip_atomic_store(f, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The value v holds in the last lane of the caller's 32-lane half.
__device__ __forceinline__ float last_of_half(float v) {
  const float lo = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 31));
  const float hi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
  return (threadIdx.x & 32) ? hi : lo;
}

// (hi, lo) += (b_hi, b_lo) with an error-free two-sum of the high parts.
__device__ __forceinline__ void add2(float& hi, float& lo, float b_hi, float b_lo) {
  float s_, e_;
  two_sum(hi, b_hi, s_, e_);
  hi = s_;
  lo = lo + (b_lo + e_);
}

// The controls the chain reads for step t of a sample from its noise e: the clamped
// g(v) (network; v = u + eps, or eps for an exploration sample) into v2 = myV + 2t, or the
// basis model's control-only terms into b8 = myB + 8t.
template <int MODEL>
__device__ __forceinline__ void step_controls(const RolloutArgs& a, float u0, float u1, float e0, float e1, bool zm,
                                              float* v2, float* b8) {
  const float vc0 = fminf(fmaxf(zm ? e0 : u0 + e0, a.u_lo0), a.u_hi0);
  const float vc1 = fminf(fmaxf(zm ? e1 : u1 + e1, a.u_lo1), a.u_hi1);
  if constexpr (MODEL == kModelNet) {
    v2[0] = vc0;
    v2[1] = vc1;
  } else {
    // {sin u_delta, -tan u_delta, u_delta, 0} and, per output o, Theta[1][o] u_F
    // + Theta[9][o] sin u_delta + Theta[24][o] u_F^2 + Theta[25][o] u_F^3
    const float sd = sinf(vc0);
    const float ntd = -tanf(vc0);
    const float w2 = vc1 * vc1, w3 = vc1 * w2;
    float c[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      float acc = a.params[0 * 4 + o] * vc1;
      acc = __builtin_fmaf(a.params[8 * 4 + o], sd, acc);
      acc = __builtin_fmaf(a.params[23 * 4 + o], w2, acc);
      c[o] = __builtin_fmaf(a.params[24 * 4 + o], w3, acc);
    }
    *reinterpret_cast<float4*>(b8) = make_float4(sd, ntd, vc0, 0.0f);
    *reinterpret_cast<float4*>(b8 + 4) = make_float4(c[0], c[1], c[2], c[3]);
  }
}

// Every block draws the noise of all its samples and steps for iteration `iter` into sE
// (one (slot, t) pair per thread at a time).
__device__ __forceinline__ void draw_block_noise(const RolloutArgs& a, uint32_t iter, int kb, int T, int eStride,
                                                 float* sE) {
  NoiseKey nk = a.nk;
  nk.iter = iter;
  for (int i = threadIdx.x; i < kWaveSlots * T; i += kSplitBlock) {
    const int slot = i / T, t = i - slot * T;
    float e0, e1;
    // the two-instruction products (philox10<false>): with them this kernel's chain loop
    // lands on a 64-byte boundary (33.7 against 34.8 us per paper-shaped step with the
    // one-instruction form, whose only effect here is where the loop lands; aligning
    // every loop instead cost 0.3 us in the padding of the others)
    draw_eps<false>((uint32_t)t, (uint32_t)(kb + slot), nk, e0, e1);
    sE[slot * eStride + 2 * t] = e0;
    sE[slot * eStride + 2 * t + 1] = e1;
  }
}

// A word that blocks of a multi-step launch poll, written through to the device's point
// of coherence.
__device__ __forceinline__ void store_word(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait of wave 0 (all 64 lanes call it) until each of the n words w[0..n)
// (n <= 64), written by other blocks with store_word, holds `target` or a later step
// (wrapping comparison): at most `limit` polls; false when they ran out.  The same in
// every lane.
__device__ __forceinline__ bool wait_words(const unsigned* w, int n, unsigned target, unsigned limit) {
  const int lane = threadIdx.x & 63;
  for (unsigned i = 0; i < limit; ++i) {
    const unsigned v = lane < n ? __hip_atomic_load(w + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : target;
    if (__all((int)(v - target) >= 0)) return true;
    __builtin_amdgcn_s_sleep(1);
  }
  return false;
}

}  // namespace

// The launch's arguments, read again at each step of a multi-step launch from the kernel
// argument segment (the kernel's one explicit argument sits at its start) through a
// pointer the compiler cannot see through: otherwise every field would be held in
// scalar registers over all steps, and the surplus spilled to vector lanes and read back
// in every phase of every step.  Valid only in code inlined into the kernel: in a function
// the kernel calls, the kernel argument segment pointer reads as null.
__device__ __forceinline__ const RolloutArgs& reload_args() {
  uint64_t v = (uint64_t)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(v));
  return *(const RolloutArgs*)(const __attribute__((address_space(4))) RolloutArgs*)v;
}

constexpr int kStatusTimeout = 6;   // a multi-step launch gave up waiting for another block

// Polls of one wait in a multi-step launch before the block gives up (0 in the arguments:
// 1 << 20: each poll waits for its load, so of the order of a second).
__device__ __forceinline__ unsigned spin_limit(const RolloutArgs& a) { return a.spin_limit ? a.spin_limit : (1u << 20); }

// Multi-step launch, merger block of group grp = blockIdx.x - G: at every step, waits
// (bounded) until the arrival word of each of the group's n_in rollout blocks shows the
// step, merges their rows into this step's group row (two buffers, alternating by step: a
// slow block may still read step s's group rows while step s + 1's are written), and
// writes the step into every copy of the group's signal word.  Inlined into the kernel,
// since it reads the arguments with reload_args().
__device__ __forceinline__ void merge_group_rows(int n_steps, float* lds) {
  __shared__ float s_small[2 * kMergeChunk];
  __shared__ unsigned s_stop;
  const int tid = threadIdx.x;
  for (int step = 0; step < n_steps; ++step) {
    const RolloutArgs& as = reload_args();
    const int T2 = 2 * as.T, stride = 2 + T2;
    const int gsz = merge_group_size(as.G);
    const int ngrp = (as.G + gsz - 1) / gsz;
    const int grp = (int)blockIdx.x - as.G;
    const int n_in = min(gsz, as.G - grp * gsz);
    const unsigned target = as.step_base + (unsigned)step + 1u;
    if (tid < 64) {
      const bool ok = wait_words(as.sync + kArriveOffset + grp * gsz, n_in, target, spin_limit(as));
      if (tid == 0) {
        if (!ok) __hip_atomic_store(as.status, kStatusTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_stop = ok ? 0u : 1u;
      }
    }
    __syncthreads();
    if (s_stop) return;
    float rho, eta;
    merge_rows<kSplitBlock>(as.part + (size_t)grp * gsz * stride, n_in, stride, T2, as.inv_lambda, lds, s_small,
                            rho, eta);
    __syncthreads();
    if (tid < 64) {
      // the group row is written through and its stores complete before the signal words
      float* dst = as.part2 + ((size_t)(step & 1) * ngrp + grp) * stride;
      if (tid == 0) {
        store_through(dst, rho);
        store_through(dst + 1, eta);
      }
      for (int o = tid; o < T2; o += 64) store_through(dst + 2 + o, lds[o]);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      if (tid < kSignalCopies) store_word(as.sync + tid * kSignalSpacing + grp, target);
    }
    __syncthreads();
  }
}

template <int MODEL, bool MULTI>
__global__ __launch_bounds__(kSplitBlock) void rollout_wave_split_kernel(RolloutArgs a) {
  constexpr int HID = 32;
  constexpr bool kNet = MODEL == kModelNet;
  extern __shared__ float smem[];
  __shared__ unsigned s_abort;
  __shared__ float s_xn[kStateDim];                  // multi-step: the next step's plant state
  __shared__ float s_small[2 * kMergeChunk];         // multi-step: the merge's row scales
  const int T = a.T;
  const int T4 = (T + 4) & ~3;
  const int eStride = (2 * T + 3) & ~3;
  const int nch = (T + 31) >> 5;                     // chunks of up to 32 steps (at most 4)
  const int r0 = T - 32 * (nch - 1);                 // steps in chunk 0 (1..32); every later chunk has 32
  const int n_steps = MULTI && a.n_steps > 1 ? a.n_steps : 1;
  float* sU = smem;                                  // [2T]
  float* sE = sU + eStride;                          // [8][2T] noise
  float* sV = sE + kWaveSlots * eStride;             // network: [8][2T] clamped controls
  float* sX = sV + (kNet ? kWaveSlots * eStride : 0);    // [8][T4][8]: hi_t, y_t
  unsigned* sFlag = reinterpret_cast<unsigned*>(sX + kWaveSlots * T4 * 8);   // [4] chain progress, [4] spare
  float* sS = reinterpret_cast<float*>(sFlag + 8);   // [8] costs
  float* sB = sS + 8;                                // basis model: [8][T][8] control terms
  float* sP = sB + (kNet ? 0 : kWaveSlots * T * 8);  // multi-step: the model's parameters (the plant step)
  // after both roles: the block's N row (the clamped controls or the basis terms are no
  // longer read) and the merge's working row (the states are no longer read)
  float* N_lds = kNet ? sV : sB;
  float* lds = sX;
  if constexpr (MULTI) {
    if ((int)blockIdx.x >= a.G) {   // a merger block (blocks G .. G + ngrp - 1)
      merge_group_rows(n_steps, sX);
      return;
    }
  }

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const bool chain = wv < kSplitPairs;
  const int pair = wv & (kSplitPairs - 1);
  const int half = lane >> 5;
  const int c32 = lane & 31;
  const int r = c32 >> 4;
  const int col = lane & 15;
  const int comp = lane & 3;
  const int slot = pair * 2 + half;
  const int kb = blockIdx.x * kWaveSlots;
  const int k = kb + slot;
  const bool valid = k < a.K;
  const bool zm = k >= a.K_imp;   // exploration sample: v = eps, delta = eps - u
  float* myE = sE + slot * eStride;
  float* myV = sV + slot * eStride;
  float* myB = sB + slot * T * 8;
  float* myX = sX + slot * T4 * 8;
  unsigned* chainCnt = sFlag + pair;

  // ---- the chain's network constants, kept in registers over every step -------------
  const float* W1 = a.params;
  const float* b1 = W1 + HID * 6;
  const float* W2 = b1 + HID;
  const float* b2 = W2 + HID * HID;
  const float* W3 = b2 + HID;
  const float* b3 = W3 + 4 * HID;
  const int j = 16 * r + col;
  const bool cn = chain && kNet;
  // layers 1 and 2 form tanh's argument already multiplied by 2 log2(e)
  float w1[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) w1[i] = cn ? kTanhScale * W1[j * 6 + i] : 0.0f;
  const float bb1 = cn ? kTanhScale * b1[j] : 0.0f;
  float wP[16], wQ[16];
  int src[16];
  src[0] = col;
  src[1] = ror_src<1>(col);   src[2] = ror_src<2>(col);   src[3] = ror_src<3>(col);
  src[4] = ror_src<4>(col);   src[5] = ror_src<5>(col);   src[6] = ror_src<6>(col);
  src[7] = ror_src<7>(col);   src[8] = ror_src<8>(col);   src[9] = ror_src<9>(col);
  src[10] = ror_src<10>(col); src[11] = ror_src<11>(col); src[12] = ror_src<12>(col);
  src[13] = ror_src<13>(col); src[14] = ror_src<14>(col); src[15] = ror_src<15>(col);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    wP[q] = cn ? kTanhScale * W2[col * HID + 16 * r + src[q]] : 0.0f;
    wQ[q] = cn ? kTanhScale * W2[(16 + col) * HID + 16 * r + src[q]] : 0.0f;
  }
  const float bP = (cn && r == 0) ? kTanhScale * b2[col] : 0.0f;
  const float bQ = (cn && r == 1) ? kTanhScale * b2[16 + col] : 0.0f;
  // layer 3 times dt as a reduce-scatter over each quad (see the wave kernel)
  const float wKA = cn ? a.dt * W3[comp * HID + j] : 0.0f;
  const float wKB = cn ? a.dt * W3[(comp ^ 2) * HID + j] : 0.0f;
  const float wSA = cn ? a.dt * W3[(comp ^ 1) * HID + j] : 0.0f;
  const float wSB = cn ? a.dt * W3[(comp ^ 3) * HID + j] : 0.0f;
  const float bKA = (cn && c32 < 4) ? a.dt * b3[comp] : 0.0f;
  // basis-function model: this lane's column of Theta with each normaliser folded in
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
  for (int i = 0; i < kRaw; ++i) kc[i] = (chain && !kNet) ? a.params[kRawIdx[i] * 4 + comp] * kRawScale[i] : 0.0f;

  const uint32_t iter0 = a.iter_dev ? *a.iter_dev : a.nk.iter;   // the device counter, advanced by the final merge
  if (tid < 2 * kSplitPairs) sFlag[tid] = 0u;
  if (tid == 0) s_abort = 0u;
  if constexpr (MULTI)   // the plant step's copy of the parameters (a network in its plant layout)
    for (int i = tid; i < (kNet ? kSplitParams : kSplitBasisParams); i += kSplitBlock)
      sP[kNet ? plant_layout_index(i, HID) : i] = a.params[i];
  // four no-ops, once per launch: they move the chain loop below onto a 64-byte boundary
  // (where the loop lands is worth ~1 us per paper-shaped step; see draw_block_noise)
  if constexpr (MULTI) asm volatile("s_nop 0\n\ts_nop 0\n\ts_nop 0\n\ts_nop 0");
  draw_block_noise(a, iter0, kb, T, eStride, sE);
  if (chain) __builtin_amdgcn_s_setprio(2);

  for (int step = 0; step < n_steps; ++step) {
    const RolloutArgs& as = MULTI ? reload_args() : a;
    // this step's counter word and history entries
    const uint32_t iter = iter0 + (uint32_t)step;
    float* const u0_out = (as.u0_out && MULTI) ? as.u0_out + 2 * step : as.u0_out;
    float* const x_copy = (as.x_copy && MULTI) ? as.x_copy + kStateDim * step : as.x_copy;
    // ---- this step's U and plant state: from global memory at the first step, from the
    // block's own final stage of the previous step after that ------------------------------
    if (step == 0)
      for (int i = tid; i < 2 * T; i += kSplitBlock) sU[i] = as.U[i];
    float x0v[kStateDim];
#pragma unroll
    for (int i = 0; i < kStateDim; ++i) x0v[i] = step > 0 ? s_xn[i] : (as.x0_dev ? as.x0_dev[i] : as.x0[i]);
    __syncthreads();
    // the controls of every sample and step; the state entry 0 of every sample
    for (int i = tid; i < kWaveSlots * T; i += kSplitBlock) {
      const int sl = i / T, t = i - sl * T;
      step_controls<MODEL>(as, sU[2 * t], sU[2 * t + 1], sE[sl * eStride + 2 * t], sE[sl * eStride + 2 * t + 1],
                           kb + sl >= as.K_imp, sV + sl * eStride + 2 * t, sB + sl * T * 8 + 8 * t);
    }
    if (tid < kWaveSlots * 4) sX[(tid >> 2) * T4 * 8 + (tid & 3)] = x0v[3 + (tid & 3)];
    __syncthreads();

    if (chain) {
      // ---- chain wave ----------------------------------------------------------------
      float xh = x0v[3 + comp];   // hi_t of the lane's component
      float2 vc = make_float2(0.0f, 0.0f);
      float4 bq = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      float cq = 0.0f;
      if constexpr (kNet) {
        vc = *reinterpret_cast<const float2*>(myV);
      } else {
        bq = *reinterpret_cast<const float4*>(myB);
        cq = myB[4 + comp];
      }
      // the lane's store slot: hi_{t+1} (lanes with bit 2 clear) or y_t (bit 2 set)
      float* xs = myX + ((lane & 4) ? 4 + comp : 8 + comp);
      for (int c = 0; c < nch; ++c) {
        const int t1 = r0 + 32 * c;
        for (int t = c > 0 ? t1 - 32 : 0; t < t1; ++t) {
          const int tn = min(t + 1, T - 1);
          float y;   // dt * f of the lane's component
          if constexpr (MODEL == kModelBasis) {
            const float4 bq_next = *reinterpret_cast<const float4*>(myB + 8 * tn);
            const float cq_next = myB[8 * tn + 4 + comp];
            const float roll = dpp_f<0x00>(xh), vx = dpp_f<0x55>(xh);   // quad_perm:[i,i,i,i]
            const float vy = dpp_f<0xAA>(xh), om = dpp_f<0xFF>(xh);
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
            y = as.dt * ((p0 + p1) + (p2 + p3));
            bq = bq_next;
            cq = cq_next;
          } else {
            const float2 vc_next = *reinterpret_cast<const float2*>(myV + 2 * tn);
            // layer 1
            float acc1 = __builtin_fmaf(w1[4], vc.x, bb1);
            acc1 = __builtin_fmaf(w1[5], vc.y, acc1);
            // the DPP source xh was written before the two fmas of acc1 above: the two
            // wait states a DPP read of a VALU result needs, so no s_nop here
            asm volatile(
                "v_fmac_f32_dpp %0, %1, %2 quad_perm:[0,0,0,0] row_mask:0xf bank_mask:0xf\n\t"
                "v_fmac_f32_dpp %0, %1, %3 quad_perm:[1,1,1,1] row_mask:0xf bank_mask:0xf\n\t"
                "v_fmac_f32_dpp %0, %1, %4 quad_perm:[2,2,2,2] row_mask:0xf bank_mask:0xf\n\t"
                "v_fmac_f32_dpp %0, %1, %5 quad_perm:[3,3,3,3] row_mask:0xf bank_mask:0xf"
                : "+v"(acc1) : "v"(xh), "v"(w1[0]), "v"(w1[1]), "v"(w1[2]), "v"(w1[3]));
            const float h1 = tanh_prescaled(acc1);
            // layer 2: four interleaved chains over the row's rotations, then the two rows
            float P = __builtin_fmaf(wP[0], h1, bP);
            float Q = __builtin_fmaf(wQ[0], h1, bQ);
            float P2 = wP[1] * dpp_f<kRowRor + 1>(h1);
            float Q2 = wQ[1] * dpp_f<kRowRor + 1>(h1);
            // the DPP source h1 precedes the four instructions forming P, Q, P2 and Q2,
            // the block's inputs: no s_nop needed (removing it saved 0.7 us per step)
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
            swap_rows(P, Q);
            const float h2 = tanh_prescaled(P + Q);
            // layer 3 (times dt)
            const float A = __builtin_fmaf(wKA, h2, bKA) + dpp_f<kQuadXor1>(wSA * h2);
            const float B = wKB * h2 + dpp_f<kQuadXor1>(wSB * h2);
            float g = A + dpp_f<kQuadXor2>(B);
            g = g + dpp_f<kRowRor + 8>(g);
            g = g + dpp_f<kRowRor + 4>(g);
            y = add_rows(g);
            vc = vc_next;
          }
          xh = xh + y;
          xs[8 * t] = (lane & 4) ? y : xh;   // y_t at entry t, hi_{t+1} at entry t + 1
        }
        publish_count(chainCnt, (unsigned)(step * nch + c + 1));
      }
    } else {
      // ---- cost wave -----------------------------------------------------------------
      if (as.ckpt && valid && c32 < kStateDim)
        as.ckpt[(size_t)k * (T / as.ckpt_every + 1) * kCkptStride + c32] = x0v[c32];
      // carries from chunk to chunk: the compensation lo of each x_d component, the
      // heading and the position (hi, lo), the cost (hi, lo)
      float lo[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      float th_h = x0v[2], th_l = 0.0f;
      float px_h = x0v[0], px_l = 0.0f, py_h = x0v[1], py_l = 0.0f;
      Acc Sacc{0.0f, 0.0f};
      bool ok = true;
      for (int c = 0; c < nch; ++c) {
        wait_count(chainCnt, (unsigned)(step * nch + c + 1));
        const int t = (c > 0 ? r0 + 32 * (c - 1) : 0) + c32;
        const bool live = c > 0 || c32 < r0;
        const int tc = min(t, T - 1);
        const float4 hv = live ? *reinterpret_cast<const float4*>(myX + 8 * tc) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const float4 yv = live ? *reinterpret_cast<const float4*>(myX + 8 * tc + 4) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        // compensated states before (xp) and after (xn) step t
        const float hq[4] = {hv.x, hv.y, hv.z, hv.w};
        const float yq[4] = {yv.x, yv.y, yv.z, yv.w};
        float xp[4], xn[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float s_, e_;
          two_sum(hq[i], yq[i], s_, e_);
          const float ex = scan32_excl(e_, c32);
          const float lt = lo[i] + ex;                 // lo_t
          xp[i] = hq[i] + lt;
          xn[i] = s_ + (lt + e_);
          lo[i] = lo[i] + last_of_half(ex + e_);       // the chunk's errors
        }
        // heading before the step: theta_0 + dt * (sum of the previous steps' theta_dot)
        const float dth = live ? as.dt * xp[3] : 0.0f;
        float sh = dth, sl = 0.0f;
        scan32_excl2(sh, sl, c32);
        float th = th_h, thl = th_l;
        add2(th, thl, sh, sl);                         // theta_t
        {
          float ih = sh, il = sl;                      // the chunk's total
          add2(ih, il, dth, 0.0f);
          add2(th_h, th_l, last_of_half(ih), last_of_half(il));
        }
        // position after the step: p_0 + dt * (sum over s <= t of R(theta_s) v_s)
        float sn, cs;
        sincosf(th + thl, &sn, &cs);
        const float dpx = live ? as.dt * (cs * xp[1] - sn * xp[2]) : 0.0f;
        const float dpy = live ? as.dt * (sn * xp[1] + cs * xp[2]) : 0.0f;
        float qxh = dpx, qxl = 0.0f, qyh = dpy, qyl = 0.0f;
        scan32_excl2(qxh, qxl, c32);
        scan32_excl2(qyh, qyl, c32);
        add2(qxh, qxl, dpx, 0.0f);                     // inclusive
        add2(qyh, qyl, dpy, 0.0f);
        float pxh = px_h, pxl = px_l, pyh = py_h, pyl = py_l;
        add2(pxh, pxl, qxh, qxl);
        add2(pyh, pyl, qyh, qyl);
        add2(px_h, px_l, last_of_half(qxh), last_of_half(qxl));
        add2(py_h, py_l, last_of_half(qyh), last_of_half(qyl));
        float th1h = th, th1l = thl;
        add2(th1h, th1l, dth, 0.0f);
        const float th1 = th1h + th1l;
        // cost of the post-step state and the control cost of the step
        int idx[4];
        float fx, fy;
        map_taps(as.cost, pxh, pxl, pyh, pyl, idx, fx, fy);
        const float mv[4] = {as.map[idx[0]], as.map[idx[1]], as.map[idx[2]], as.map[idx[3]]};
        const float dec = as.decay[tc + 1];
        if (live) {
          const float px1 = pxh + pxl, py1 = pyh + pyl;
          if (as.ckpt && ((t + 1) % as.ckpt_every) == 0 && valid) {
            float* cp = as.ckpt + ((size_t)k * (T / as.ckpt_every + 1) + (t + 1) / as.ckpt_every) * kCkptStride;
            cp[0] = px1; cp[1] = py1; cp[2] = th1;
            cp[3] = xn[0]; cp[4] = xn[1]; cp[5] = xn[2]; cp[6] = xn[3];
          }
          Sacc.add(state_cost_h(as.cost, bilerp(mv, fx, fy), dec, xn[1], xn[2]));
          const float u0 = sU[2 * t], u1 = sU[2 * t + 1];
          const float d0 = zm ? myE[2 * t] - u0 : myE[2 * t];
          const float d1 = zm ? myE[2 * t + 1] - u1 : myE[2 * t + 1];
          Sacc.add(as.gcs0 * (u0 * d0) + as.gcs1 * (u1 * d1));
          ok = ok && finite_f(px1) && finite_f(py1) && finite_f(th1) && finite_f(xn[0]) && finite_f(xn[1]) &&
               finite_f(xn[2]) && finite_f(xn[3]);
          if (as.cem_zeta > 0 && valid) {
            float* drow = as.D + (size_t)k * 2 * T;
            drow[2 * t] = d0;
            drow[2 * t + 1] = d1;
          }
        }
      }
      float S_h = Sacc.hi, S_l = Sacc.lo;
      sum32_2(S_h, S_l);
      float S = S_h + S_l;
      if (!valid || !all32(ok) || !finite_f(S)) S = kInf;
      if (valid && c32 == 0) store_through(as.S + k, S);   // read by the host or Algorithm 3's update
      if (c32 == 0) sS[slot] = S;
    }
    __syncthreads();
    if (as.cem_zeta > 0) return;   // the cross-entropy update runs in the launch that follows

    // ---- the block's softmin partial (rho_g, eta_g, N_g) ------------------------------
    float Sk[kWaveSlots];
#pragma unroll
    for (int q = 0; q < kWaveSlots; ++q) Sk[q] = sS[q];
    float rho = Sk[0];
#pragma unroll
    for (int q = 1; q < kWaveSlots; ++q) rho = fminf(rho, Sk[q]);
    float wgt[kWaveSlots];
    float eta = 0.0f;
#pragma unroll
    for (int q = 0; q < kWaveSlots; ++q) {
      wgt[q] = rel_weight(Sk[q], rho, as.inv_lambda);
      eta += wgt[q];
    }
    for (int o = tid; o < 2 * T; o += kSplitBlock) {
      const float u = sU[o];
      float n = 0.0f;
#pragma unroll
      for (int q = 0; q < kWaveSlots; ++q) {
        const float e = sE[q * eStride + o];
        n = __builtin_fmaf(wgt[q], (kb + q >= as.K_imp) ? e - u : e, n);
      }
      N_lds[o] = n;
    }
    if constexpr (MULTI) {
      // ---- multi-step launch: the row goes to the group's merger block; this block then
      // merges the group rows and runs the final stage itself ---------------------------
      const int T2 = 2 * T, stride = 2 + T2;
      const int gsz = merge_group_size(as.G);
      const int ngrp = (as.G + gsz - 1) / gsz;
      const unsigned target = as.step_base + (unsigned)step + 1u;
      FinalStage<kSplitBlock, MODEL, true, HID, kNet> fs;
      fs.prefetch_local(as, sU, x0v);
      __syncthreads();   // the block's N row is complete
      if (tid < 64) {
        // the row is written through and its stores complete before the arrival word
        float* dst = as.part + (size_t)blockIdx.x * stride;
        if (tid == 0) {
          store_through(dst, rho);
          store_through(dst + 1, eta);
        }
        for (int o = tid; o < T2; o += 64) store_through(dst + 2 + o, N_lds[o]);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if (tid == 0) store_word(as.sync + kArriveOffset + blockIdx.x, target);
      }
      // the next step's noise does not depend on its U: drawn while the merges complete
      if (step + 1 < n_steps) draw_block_noise(as, iter + 1u, kb, T, eStride, sE);
      if (tid < 64) {
        const bool ok = wait_words(as.sync + (blockIdx.x % kSignalCopies) * kSignalSpacing, ngrp, target,
                                   spin_limit(as));
        if (tid == 0 && !ok) {
          s_abort = 1u;
          __hip_atomic_store(as.status, kStatusTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      __syncthreads();
      if (s_abort) break;
      float rho_m, eta_m;
      merge_rows<kSplitBlock>(as.part2 + (size_t)(step & 1) * ngrp * stride, ngrp, stride, T2, as.inv_lambda, lds,
                              s_small, rho_m, eta_m);
      const bool fin = (rho_m < kInf) && (eta_m > 0.0f);
      fs.apply(as, lds, fin, fin ? 1.0f / eta_m : 0.0f, sP, rho_m, fin ? eta_m : 0.0f, iter, u0_out, x_copy,
               blockIdx.x == 0, sU, s_xn);
      __syncthreads();   // the next step's U (sU) and plant state (s_xn)
    } else {
      const StepTarget target{iter, u0_out, x_copy};
      finish_iteration<kSplitBlock, MODEL, true, HID>(as, blockIdx.x, rho, eta, N_lds, lds, as.params, &target);
    }
  }
}

template __global__ void rollout_wave_split_kernel<kModelNet, false>(RolloutArgs);
template __global__ void rollout_wave_split_kernel<kModelBasis, false>(RolloutArgs);
template __global__ void rollout_wave_split_kernel<kModelNet, true>(RolloutArgs);
template __global__ void rollout_wave_split_kernel<kModelBasis, true>(RolloutArgs);

// Dynamic LDS bytes of the split kernel for horizon T (T <= 128).
size_t wave_split_smem_bytes(int T, int model) {
  const size_t e = (size_t)((2 * T + 3) & ~3);
  const size_t T4 = (size_t)((T + 4) & ~3);
  const size_t v = model == kModelNet ? (size_t)kWaveSlots * e : 0;
  const size_t basis = model == kModelBasis ? (size_t)kWaveSlots * T * 8 : 0;
  return sizeof(float) * (e + kWaveSlots * e + v + (size_t)kWaveSlots * T4 * 8 + 8 + 8 + basis + kSplitParams);
}

}  // namespace mppi
