// Device-side primitives of the MPPI kernels (gfx950).
//
//  * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11),
//    counter (t, k, iter, instance) with k the global sample index, key (seed_lo, seed_hi).
//  * Box-Muller transform (Box & Muller 1958) on the first two words, with this
//    project's FP32 log (exponent split + atanh series) and quadrant-reduced
//    sin/cos (Taylor series in (pi/2) r); every operation is an IEEE single
//    operation or an explicit fma, so the draws are reproducible bit for bit.
//  * tanh for the dynamics network, the bilinear cost-map lookup and the state
//    cost of the paper's Section VI-C.
//
// Compiled with -ffp-contract=off: fused multiply-adds appear only where written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mppi_types.h"

namespace mppi {

// ---------------------------------------------------------------------------
// Philox4x32-10
// ---------------------------------------------------------------------------
struct U32x4 {
  uint32_t x, y, z, w;
};

// WIDE: each round's 32 x 32 -> 64-bit products as one v_mad_u64_u32 each (~30 % more
// Philox calls per second on gfx950 than a v_mul_lo_u32 and a v_mul_hi_u32 each); the
// same words either way.
template <bool WIDE = true>
__device__ __forceinline__ U32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo_a, hi_a, lo_b, hi_b;
    if constexpr (WIDE) {
      const uint64_t pa = (uint64_t)c0 * 0xD2511F53u;
      const uint64_t pb = (uint64_t)c2 * 0xCD9E8D57u;
      lo_a = (uint32_t)pa;
      hi_a = (uint32_t)(pa >> 32);
      lo_b = (uint32_t)pb;
      hi_b = (uint32_t)(pb >> 32);
    } else {
      lo_a = c0 * 0xD2511F53u;
      hi_a = __umulhi(c0, 0xD2511F53u);
      lo_b = c2 * 0xCD9E8D57u;
      hi_b = __umulhi(c2, 0xCD9E8D57u);
    }
    const uint32_t y0 = hi_b ^ c1 ^ k0;
    const uint32_t y2 = hi_a ^ c3 ^ k1;
    c0 = y0;
    c1 = lo_b;
    c2 = y2;
    c3 = lo_a;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U32x4{c0, c1, c2, c3};
}

// ---------------------------------------------------------------------------
// Noise transform.  A 32-bit word w gives the odd integer n = 2*(w>>9)+1 < 2^24
// and the uniform u = n * 2^-24 in (0, 1), exact in FP32.
// ---------------------------------------------------------------------------

// ln u.  n = 2^e f with f in [1, 2), halved once more when f >= fl32(sqrt 2);
// ln f = 2 atanh(s), s = (f-1)/(f+1), atanh s = s + (s z) P(z), z = s^2,
// P(z) = 1/3 + z/5 + z^2/7 + z^3/9 + z^4/11 (FP32 coefficients, Horner with fma).
__device__ __forceinline__ float noise_ln(uint32_t w) {
  const uint32_t n = ((w >> 9) << 1) | 1u;
  int e = 31 - __builtin_clz(n);
  float f = __builtin_ldexpf((float)n, -e);
  if (f >= 0x1.6a09e6p+0f) {
    f = f * 0.5f;
    e += 1;
  }
  const float s = (f - 1.0f) / (f + 1.0f);
  const float z = s * s;
  float p = 0x1.745d18p-4f;          // 1/11
  p = __builtin_fmaf(p, z, 0x1.c71c72p-4f);   // 1/9
  p = __builtin_fmaf(p, z, 0x1.24924ap-3f);   // 1/7
  p = __builtin_fmaf(p, z, 0x1.99999ap-3f);   // 1/5
  p = __builtin_fmaf(p, z, 0x1.555556p-2f);   // 1/3
  const float at = __builtin_fmaf(s * z, p, s);
  return __builtin_fmaf((float)(e - 24), 0x1.62e430p-1f, 2.0f * at);   // + (e-24) ln 2
}

// cos(2 pi u), sin(2 pi u).  2 pi u = (pi/2)(q + r): q = nearest quadrant from the
// integer n, r = (n - q 2^22) 2^-22 in (-1/2, 1/2), exact.  sin((pi/2) r) to r^11 and
// cos((pi/2) r) to r^12, coefficients (-1)^j (pi/2)^m / m! in FP32, Horner in r^2.
__device__ __forceinline__ void noise_cs(uint32_t w, float& c_out, float& s_out) {
  const uint32_t n = ((w >> 9) << 1) | 1u;
  const uint32_t q = (n + (1u << 21)) >> 22;
  const int32_t rr = (int32_t)n - (int32_t)(q << 22);
  const float r = __builtin_ldexpf((float)rr, -22);
  const float r2 = r * r;
  float ps = -0x1.e30750p-19f;                    // m = 11
  ps = __builtin_fmaf(ps, r2, 0x1.507834p-13f);   // m = 9
  ps = __builtin_fmaf(ps, r2, -0x1.32d2ccp-8f);   // m = 7
  ps = __builtin_fmaf(ps, r2, 0x1.466bc6p-4f);    // m = 5
  ps = __builtin_fmaf(ps, r2, -0x1.4abbcep-1f);   // m = 3
  ps = __builtin_fmaf(ps, r2, 0x1.921fb6p+0f);    // m = 1
  const float sn = r * ps;
  float pc = 0x1.f9d38ap-22f;                     // m = 12
  pc = __builtin_fmaf(pc, r2, -0x1.a6d1f2p-16f);  // m = 10
  pc = __builtin_fmaf(pc, r2, 0x1.e1f506p-11f);   // m = 8
  pc = __builtin_fmaf(pc, r2, -0x1.55d3c8p-6f);   // m = 6
  pc = __builtin_fmaf(pc, r2, 0x1.03c1f0p-2f);    // m = 4
  pc = __builtin_fmaf(pc, r2, -0x1.3bd3ccp+0f);   // m = 2
  const float cs = __builtin_fmaf(pc, r2, 1.0f);
  const uint32_t qq = q & 3u;
  const float a = (qq & 1u) ? sn : cs;            // |cos| candidate
  const float b = (qq & 1u) ? cs : sn;            // |sin| candidate
  c_out = (qq == 1u || qq == 2u) ? -a : a;
  s_out = (qq >= 2u) ? -b : b;
}

// eps_{k,t} for iteration `iter`: sqrt(Sigma_ii) * (R cos, R sin), R = sqrt(-2 ln u1).
// k is the launch's sample index; the counter takes the global one, nk.k_base + k.
// WIDE: see philox10.
template <bool WIDE = true>
__device__ __forceinline__ void draw_eps(uint32_t t, uint32_t k, const NoiseKey& nk, float& e0,
                                         float& e1) {
  const U32x4 r = philox10<WIDE>(t, nk.k_base + k, nk.iter, nk.instance, nk.key_lo, nk.key_hi);
  const float L = noise_ln(r.x);
  const float R = __builtin_sqrtf(-2.0f * L);
  float c, s;
  noise_cs(r.y, c, s);
  e0 = nk.sig0 * (R * c);
  e1 = nk.sig1 * (R * s);
}

// ---------------------------------------------------------------------------
// Network nonlinearity: tanh x = 1 - 2 / (2^(2x log2 e) + 1), one exp2 and one rcp
// on the transcendental unit; saturates correctly at +-inf, propagates NaN.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float tanh_f(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.88539008177792681f);
  return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

// The scale 2 log2(e) of tanh_f's argument, for kernels that fold it into the weights.
constexpr float kTanhScale = 2.88539008177792681f;

// tanh x from a = x * kTanhScale (formed by weights already multiplied by the scale).
__device__ __forceinline__ float tanh_prescaled(float a) {
  const float e = __builtin_amdgcn_exp2f(a);
  return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

// ---------------------------------------------------------------------------
// Basis-function dynamics model (appendix; Section VI-B-1)
// ---------------------------------------------------------------------------
// f(x_d, v) = Theta^T phi(x_d, v) with 25 basis functions; Theta is [25][4] row-major
// (row = basis function, column = d/dt of roll, v_x, v_y, heading rate).  The appendix
// names the heading (yaw) rate r and the roll theta; here they are x_d[3] and x_d[0].
// u_delta = steering g(v)_1, u_F = throttle g(v)_2, sd = sin(u_delta),
// td = tan(u_delta) (read only when v_x <= 0.1).  The tyre tangents tan(alpha) use
// tan(arctan z) = z: above v_x = 0.1 they are z itself, so no arctan or tan is needed.
constexpr int kNumBasis = 25;

__device__ __forceinline__ void basis_phi(float roll, float vx, float vy, float om, float uF, float sd,
                                          float td, float ud, float phi[kNumBasis]) {
  float q = 0.0f, tf, tr = 0.0f;
  if (vx > 0.1f) {
    const float rv = 1.0f / vx;
    q = vy * rv;
    tf = (q + (0.45f * om) * rv) - ud;
    tr = q - (0.35f * om) * rv;
  } else {
    tf = -td;
  }
  const float atf = fabsf(tf), atr = fabsf(tr);
  const float sf = sd * tf;
  phi[0] = uF;
  phi[1] = vx * 0.1f;
  phi[2] = sf * (1.0f / 1200.0f);
  phi[3] = (sf * atf) * (1.0f / (1200.0f * 1200.0f));
  phi[4] = (sf * (tf * tf)) * (1.0f / (1200.0f * 1200.0f * 1200.0f));
  phi[5] = (om * vy) * (1.0f / 25.0f);
  phi[6] = om * 0.1f;
  phi[7] = vy * 0.1f;
  phi[8] = sd;
  phi[9] = q * (1.0f / 40.0f);
  phi[10] = tf * (1.0f / 1400.0f);
  phi[11] = (tf * atf) * (1.0f / (1400.0f * 1400.0f));
  phi[12] = (tf * (tf * tf)) * (1.0f / (1400.0f * 1400.0f * 1400.0f));
  phi[13] = tr * (1.0f / 40.0f);
  phi[14] = (tr * atr) * (1.0f / (40.0f * 40.0f));
  phi[15] = (tr * (tr * tr)) * (1.0f / (40.0f * 40.0f * 40.0f));
  phi[16] = (om * vx) * (1.0f / 50.0f);
  phi[17] = roll;
  phi[18] = roll * om;
  phi[19] = (roll * vx) * (1.0f / 3.0f);
  phi[20] = ((roll * vx) * om) * 0.2f;
  phi[21] = (vx * vx) * 0.01f;
  phi[22] = (vx * (vx * vx)) * 0.001f;
  phi[23] = uF * uF;
  phi[24] = uF * (uF * uF);
}

// Output o of f (the sum over i of Theta[i][o] phi_i, in i order).
__device__ __forceinline__ float basis_out(const float* __restrict__ th, const float xd[4], float ud, float uF,
                                           int o) {
  const float sd = sinf(ud);
  float td = 0.0f;
  if (!(xd[1] > 0.1f)) td = tanf(ud);
  float phi[kNumBasis];
  basis_phi(xd[0], xd[1], xd[2], xd[3], uF, sd, td, ud, phi);
  float acc = 0.0f;
#pragma unroll
  for (int i = 0; i < kNumBasis; ++i) acc = __builtin_fmaf(th[i * 4 + o], phi[i], acc);
  return acc;
}

// All four outputs in one thread (the plant step and the lane schedule); each equals
// basis_out() bit for bit.
__device__ __forceinline__ void basis_f(const float* __restrict__ th, const float xd[4], float ud, float uF,
                                        float f[4]) {
  const float sd = sinf(ud);
  float td = 0.0f;
  if (!(xd[1] > 0.1f)) td = tanf(ud);
  float phi[kNumBasis];
  basis_phi(xd[0], xd[1], xd[2], xd[3], uF, sd, td, ud, phi);
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < kNumBasis; ++i) acc = __builtin_fmaf(th[i * 4 + o], phi[i], acc);
    f[o] = acc;
  }
}

// ---------------------------------------------------------------------------
// Cost map and state cost (Section VI-C)
// ---------------------------------------------------------------------------

// Bilinear lookup, cell (i, j) at world (ox + j res, oy + i res), indices clamped
// to the map edge.  The grid coordinate is clamped to [-1, W] x [-1, H] first,
// which changes nothing inside the map and keeps the integer conversion in range.
__device__ __forceinline__ float costmap_at(const CostArgs& c, const float* __restrict__ map,
                                            float px, float py) {
  float gx = (px - c.ox) / c.res;
  float gy = (py - c.oy) / c.res;
  gx = fminf(fmaxf(gx, -1.0f), (float)c.W);
  gy = fminf(fmaxf(gy, -1.0f), (float)c.H);
  const float fj = floorf(gx), fi = floorf(gy);
  const int j0 = (int)fj, i0 = (int)fi;
  const float fx = gx - fj, fy = gy - fi;
  const int ja = min(max(j0, 0), c.W - 1), jb = min(max(j0 + 1, 0), c.W - 1);
  const int ia = min(max(i0, 0), c.H - 1), ib = min(max(i0 + 1, 0), c.H - 1);
  const float m00 = map[(size_t)ia * c.W + ja];
  const float m01 = map[(size_t)ia * c.W + jb];
  const float m10 = map[(size_t)ib * c.W + ja];
  const float m11 = map[(size_t)ib * c.W + jb];
  const float top = (1.0f - fx) * m00 + fx * m01;
  const float bot = (1.0f - fx) * m10 + fx * m11;
  return (1.0f - fy) * top + fy * bot;
}

// Exact sum and its rounding error (Knuth's two-sum).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Grid coordinate (p - o) / res of a position given as hi + lo, split into an integer
// cell and a fraction in [0, 1) that keeps the low part: the quotient's rounding
// remainder is exact (fma), so the fraction is good to ~1e-7 of a cell even where
// the coordinate itself needs all 24 bits.  Clamped to [-1, n] like costmap_at.  The
// quotient comes from the reciprocal inv_res = fl(1/res) and one correction with the
// residual (within an ulp of d / res, which keeps the next residual exact), not from
// a division.
__device__ __forceinline__ void grid_coord(float ph, float pl, float o, float res, float inv_res, int n,
                                           int& i0, float& f) {
  float d, dl;
  two_sum(ph, -o, d, dl);
  dl = dl + pl;
  float q = d * inv_res;
  q = __builtin_fmaf(__builtin_fmaf(-q, res, d), inv_res, q);
  const float rem = __builtin_fmaf(-q, res, d);
  float ql = (rem + dl) * inv_res;
  if (!(q >= -1.0f)) { q = -1.0f; ql = 0.0f; }
  if (!(q <= (float)n)) { q = (float)n; ql = 0.0f; }
  const float fl = floorf(q);
  i0 = (int)fl;
  f = (q - fl) + ql;
  if (f < 0.0f) { f += 1.0f; i0 -= 1; }
  if (f >= 1.0f) { f -= 1.0f; i0 += 1; }
}

// Cell indices (row-major offsets of the four corners, clamped to the edge) and
// fractions of the bilinear lookup at a hi + lo position.
__device__ __forceinline__ void map_taps(const CostArgs& c, float pxh, float pxl, float pyh, float pyl,
                                         int idx[4], float& fx, float& fy) {
  int j0, i0;
  const float inv_res = 1.0f / c.res;
  grid_coord(pxh, pxl, c.ox, c.res, inv_res, c.W, j0, fx);
  grid_coord(pyh, pyl, c.oy, c.res, inv_res, c.H, i0, fy);
  const int ja = min(max(j0, 0), c.W - 1), jb = min(max(j0 + 1, 0), c.W - 1);
  const int ia = min(max(i0, 0), c.H - 1), ib = min(max(i0 + 1, 0), c.H - 1);
  idx[0] = ia * c.W + ja;
  idx[1] = ia * c.W + jb;
  idx[2] = ib * c.W + ja;
  idx[3] = ib * c.W + jb;
}

__device__ __forceinline__ float bilerp(const float m[4], float fx, float fy) {
  const float top = (1.0f - fx) * m[0] + fx * m[1];
  const float bot = (1.0f - fx) * m[2] + fx * m[3];
  return (1.0f - fy) * top + fy * bot;
}

__device__ __forceinline__ float costmap_at2(const CostArgs& c, const float* __restrict__ map,
                                             float pxh, float pxl, float pyh, float pyl) {
  int idx[4];
  float fx, fy;
  map_taps(c, pxh, pxl, pyh, pyl, idx, fx, fy);
  const float m[4] = {map[idx[0]], map[idx[1]], map[idx[2]], map[idx[3]]};
  return bilerp(m, fx, fy);
}

// c(x, t) given the map value h at the post-step position and fl32(decay^t).
__device__ __forceinline__ float state_cost_h(const CostArgs& c, float h, float decay_t, float vx, float vy) {
  float cost = c.w_map * h;
  if (h > c.map_thresh) cost += c.crash_cost * decay_t;
  const float dv = vx - c.v_des;
  cost += c.w_speed * (dv * dv);
  const float zeta = -atan2f(vy, fabsf(vx));
  cost += c.w_slip * (zeta * zeta);
  if (fabsf(zeta) > c.slip_thresh) cost += c.slip_cost;
  return cost;
}

// c(x, t) with the position as hi + lo pairs (see grid_coord).
__device__ __forceinline__ float state_cost2(const CostArgs& c, const float* __restrict__ map,
                                             const float* __restrict__ decay, float pxh, float pxl,
                                             float pyh, float pyl, float vx, float vy, int t) {
  const float h = costmap_at2(c, map, pxh, pxl, pyh, pyl);
  return state_cost_h(c, h, decay[t], vx, vy);
}

// c(x, t) on the post-step state: track (+ decaying impulse), speed, side slip.
__device__ __forceinline__ float state_cost(const CostArgs& c, const float* __restrict__ map,
                                            const float* __restrict__ decay, float px, float py,
                                            float vx, float vy, int t) {
  const float h = costmap_at(c, map, px, py);
  float cost = c.w_map * h;
  if (h > c.map_thresh) cost += c.crash_cost * decay[t];
  const float dv = vx - c.v_des;
  cost += c.w_speed * (dv * dv);
  const float zeta = -atan2f(vy, fabsf(vx));
  cost += c.w_slip * (zeta * zeta);
  if (fabsf(zeta) > c.slip_thresh) cost += c.slip_cost;
  return cost;
}

// Gradient of the smooth part of c(x) with respect to (p_x, p_y, v_x, v_y): the
// bilinear map's slope (zero where the lookup is clamped to the edge), the speed
// term and the slip term; the impulse indicators are piecewise constant and
// contribute nothing.
__device__ __forceinline__ void state_cost_grad(const CostArgs& c, const float* __restrict__ map,
                                                float px, float py, float vx, float vy, float& gpx,
                                                float& gpy, float& gvx, float& gvy) {
  float gx = (px - c.ox) / c.res;
  float gy = (py - c.oy) / c.res;
  gx = fminf(fmaxf(gx, -1.0f), (float)c.W);
  gy = fminf(fmaxf(gy, -1.0f), (float)c.H);
  const float fj = floorf(gx), fi = floorf(gy);
  const int j0 = (int)fj, i0 = (int)fi;
  const float fx = gx - fj, fy = gy - fi;
  const int ja = min(max(j0, 0), c.W - 1), jb = min(max(j0 + 1, 0), c.W - 1);
  const int ia = min(max(i0, 0), c.H - 1), ib = min(max(i0 + 1, 0), c.H - 1);
  const float m00 = map[(size_t)ia * c.W + ja];
  const float m01 = map[(size_t)ia * c.W + jb];
  const float m10 = map[(size_t)ib * c.W + ja];
  const float m11 = map[(size_t)ib * c.W + jb];
  gpx = c.w_map * (((1.0f - fy) * (m01 - m00) + fy * (m11 - m10)) / c.res);
  gpy = c.w_map * (((1.0f - fx) * (m10 - m00) + fx * (m11 - m01)) / c.res);
  gvx = 2.0f * c.w_speed * (vx - c.v_des);
  gvy = 0.0f;
  const float den = vx * vx + vy * vy;
  if (den > 0.0f) {
    const float zeta = -atan2f(vy, fabsf(vx));
    const float sgn = vx > 0.0f ? 1.0f : (vx < 0.0f ? -1.0f : 0.0f);
    gvx += 2.0f * c.w_slip * zeta * (vy * sgn / den);
    gvy += 2.0f * c.w_slip * zeta * (-fabsf(vx) / den);
  }
}

__device__ __forceinline__ bool finite_f(float v) { return __builtin_isfinite(v); }

// Compensated accumulator: the value is hi + lo.  add() folds in the rounding error
// of hi + y exactly (Knuth's two-sum), so a T-step accumulation keeps the error of
// one rounding instead of sqrt(T) of them.  Used for the states and for S_k.
struct Acc {
  float hi, lo;
  __device__ __forceinline__ void add(float y) {
    const float s = hi + y;
    const float bb = s - hi;
    const float err = (hi - (s - bb)) + (y - bb);
    hi = s;
    lo = lo + err;
  }
  __device__ __forceinline__ float value() const { return hi + lo; }
};

}  // namespace mppi
