// Cross-lane building blocks of the 32-lanes-per-sample layout (two samples per
// wavefront; lane = 32 * sample + 16 * row + column).  Shared by the forward
// ("wave") rollout and the adjoint rollout.
#pragma once

#include "kernels_common.hip.h"

namespace mppi {

constexpr int kWaveBlock = 256;
constexpr int kWaveSlots = 8;        // samples per block
constexpr int kWaveNT = kTMax / 32;  // chunks of 32 steps

__device__ __forceinline__ float as_f(uint32_t v) { return __builtin_bit_cast(float, v); }
__device__ __forceinline__ uint32_t as_u(float v) { return __builtin_bit_cast(uint32_t, v); }

// acc += src[dpp lane] * w, as one v_fmac_f32 with a DPP source operand.  The first
// use after src was written is preceded by two wait states (VALU write -> DPP read).
#define FMAC_DPP(acc, src, w, ctrl) \
  asm volatile("v_fmac_f32_dpp %0, %1, %2 " ctrl " row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(src), "v"(w))
#define FMAC_DPP_FIRST(acc, src, w, ctrl)                                                        \
  asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 " ctrl " row_mask:0xf bank_mask:0xf" : "+v"(acc) \
      : "v"(src), "v"(w))

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return as_f((uint32_t)__builtin_amdgcn_mov_dpp((int)as_u(v), CTRL, 0xf, 0xf, true));
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}

constexpr int kRowRor = 0x120;        // row_ror:s = 0x120 + s
constexpr int kQuadXor1 = 0xB1;       // quad_perm:[1,0,3,2]
constexpr int kQuadXor2 = 0x4E;       // quad_perm:[2,3,0,1]

// Column (0..15) whose value lane `col` reads through row_ror:S.
template <int S>
__device__ __forceinline__ int ror_src(int col) {
  return dpp_i<kRowRor + S>(col);
}

// Exchange between the two 16-lane rows of each 32-lane half: returns the pair
// (new first operand, new second operand) of v_permlane16_swap.
__device__ __forceinline__ void swap_rows(float& a, float& b) {
  auto r = __builtin_amdgcn_permlane16_swap(as_u(a), as_u(b), false, false);
  a = as_f(r[0]);
  b = as_f(r[1]);
}

// Sum of v over the sample's two rows, the same bits in both rows.
__device__ __forceinline__ float add_rows(float v) {
  float x = v, y = v;
  swap_rows(x, y);
  return x + y;
}

__device__ __forceinline__ float scan32_incl(float v, int c32) {
#pragma unroll
  for (int d = 1; d < 32; d <<= 1) {
    const float o = __shfl_up(v, d, 32);
    if (c32 >= d) v += o;
  }
  return v;
}

// Compensated exclusive scan of (hi, lo) pairs over the 32 lanes of a half-wave.
__device__ __forceinline__ void scan32_excl2(float& hi, float& lo, int c32) {
#pragma unroll
  for (int d = 1; d < 32; d <<= 1) {
    const float oh = __shfl_up(hi, d, 32);
    const float ol = __shfl_up(lo, d, 32);
    if (c32 >= d) {
      float s_, e_;
      two_sum(hi, oh, s_, e_);
      hi = s_;
      lo = lo + (ol + e_);
    }
  }
  const float ph = __shfl_up(hi, 1, 32);
  const float pl = __shfl_up(lo, 1, 32);
  hi = c32 == 0 ? 0.0f : ph;
  lo = c32 == 0 ? 0.0f : pl;
}

// Compensated sum of (hi, lo) over the 32 lanes, the same bits in every lane.
__device__ __forceinline__ void sum32_2(float& hi, float& lo) {
#pragma unroll
  for (int m = 16; m >= 1; m >>= 1) {
    const float oh = __shfl_xor(hi, m, 32);
    const float ol = __shfl_xor(lo, m, 32);
    float s_, e_;
    two_sum(hi, oh, s_, e_);
    hi = s_;
    lo = (lo + ol) + e_;
  }
}

__device__ __forceinline__ float sum32(float v) {
#pragma unroll
  for (int m = 16; m >= 1; m >>= 1) v += __shfl_xor(v, m, 32);
  return v;
}

}  // namespace mppi
