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

constexpr int kRowShr = 0x110;        // row_shr:s = 0x110 + s
constexpr int kRowBcast15 = 0x142;    // lane 15 of each row to every lane of the next row

// DPP move with a row mask: lanes of the rows in ROWMASK whose source lane exists take
// v from it; every other lane keeps `old`.
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ float dpp_upd(float old, float v) {
  return as_f((uint32_t)__builtin_amdgcn_update_dpp((int)as_u(old), (int)as_u(v), CTRL, ROWMASK, 0xF, false));
}

// One step of a compensated scan: (hi, lo) += the pair that DPP control CTRL brings in
// (lanes outside ROWMASK, or without a source lane, add (0, 0)).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ void scan_step2(float& hi, float& lo) {
  const float oh = dpp_upd<CTRL, ROWMASK>(0.0f, hi);
  const float ol = dpp_upd<CTRL, ROWMASK>(0.0f, lo);
  float s_, e_;
  two_sum(hi, oh, s_, e_);
  hi = s_;
  lo = lo + (ol + e_);
}

// Compensated exclusive scan of (hi, lo) pairs over the 32 lanes of a half-wave
// (lane 0 of each half gets (0, 0)), in DPP moves: the pairs are shifted up one lane,
// scanned within each 16-lane row (shifts 1, 2, 4, 8), and the first row's total is
// added to the second row.
__device__ __forceinline__ void scan32_excl2(float& hi, float& lo, int c32) {
  const bool col0 = (c32 & 15) == 0;
  {
    const float sh = dpp_upd<kRowShr + 1>(0.0f, hi), sl = dpp_upd<kRowShr + 1>(0.0f, lo);
    const float bh = dpp_upd<kRowBcast15, 0xA>(0.0f, hi), bl = dpp_upd<kRowBcast15, 0xA>(0.0f, lo);
    hi = col0 ? bh : sh;
    lo = col0 ? bl : sl;
  }
  scan_step2<kRowShr + 1, 0xF>(hi, lo);
  scan_step2<kRowShr + 2, 0xF>(hi, lo);
  scan_step2<kRowShr + 4, 0xF>(hi, lo);
  scan_step2<kRowShr + 8, 0xF>(hi, lo);
  scan_step2<kRowBcast15, 0xA>(hi, lo);
}

// Exclusive scan of v over the 32 lanes of a half-wave (lane 0 of each half gets 0), in
// DPP moves: shift up one lane, scan within each 16-lane row, add the first row's total
// to the second row.
__device__ __forceinline__ float scan32_excl(float v, int c32) {
  const bool col0 = (c32 & 15) == 0;
  const float sh = dpp_upd<kRowShr + 1>(0.0f, v);
  const float bh = dpp_upd<kRowBcast15, 0xA>(0.0f, v);
  v = col0 ? bh : sh;
  v = v + dpp_upd<kRowShr + 1, 0xF>(0.0f, v);
  v = v + dpp_upd<kRowShr + 2, 0xF>(0.0f, v);
  v = v + dpp_upd<kRowShr + 4, 0xF>(0.0f, v);
  v = v + dpp_upd<kRowShr + 8, 0xF>(0.0f, v);
  v = v + dpp_upd<kRowBcast15, 0xA>(0.0f, v);
  return v;
}

// Compensated sum of (hi, lo) over the 32 lanes, the same bits in every lane (the
// error-free two-sum is symmetric in its operands): butterflies within each row, then
// the two rows.
__device__ __forceinline__ void sum32_2(float& hi, float& lo) {
  auto step = [&](float oh, float ol) {
    float s_, e_;
    two_sum(hi, oh, s_, e_);
    hi = s_;
    lo = (lo + ol) + e_;
  };
  step(dpp_f<kRowRor + 8>(hi), dpp_f<kRowRor + 8>(lo));
  step(dpp_f<kRowRor + 4>(hi), dpp_f<kRowRor + 4>(lo));
  step(dpp_f<kQuadXor2>(hi), dpp_f<kQuadXor2>(lo));
  step(dpp_f<kQuadXor1>(hi), dpp_f<kQuadXor1>(lo));
  float xh = hi, yh = hi, xl = lo, yl = lo;
  swap_rows(xh, yh);
  swap_rows(xl, yl);
  // each lane now holds its own row's (hi, lo) in one operand and the other row's in the other
  const bool r1 = (threadIdx.x & 16) != 0;
  hi = r1 ? yh : xh;
  lo = r1 ? yl : xl;
  step(r1 ? xh : yh, r1 ? xl : yl);
}

// The value of v in the lane 32 apart (the other half of the wave).
__device__ __forceinline__ float other_half(float v) {
  auto r = __builtin_amdgcn_permlane32_swap(as_u(v), as_u(v), false, false);
  // r[0] holds the first half's values in both halves, r[1] the second half's
  return as_f((threadIdx.x & 32) ? r[0] : r[1]);
}

// Whether p holds in every lane of the calling lane's 32-lane half.
__device__ __forceinline__ bool all32(bool p) {
  const unsigned long long m = __ballot(p);
  const unsigned half = (threadIdx.x & 32) ? (unsigned)(m >> 32) : (unsigned)m;
  return half == 0xFFFFFFFFu;
}

}  // namespace mppi
