// MPPI / information-theoretic MPC reference oracle: a plain, slow, CPU-only
// implementation of one iteration of the paper's sampling-based MPC
// (Williams et al., "Information Theoretic Model Predictive Control: Theory and
// Applications to Autonomous Driving", arXiv 1707.02342).
//
// TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
// checked against.  Nothing in the product path may link, load or call it;
// only the tests, the smoke check and the benchmark's CPU-baseline leg do.
// It shares no code, header, table or constant generator with the GPU library.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread
// (no contraction, IEEE division and square root: the noise transform below
// must be bit-identical with the independent GPU implementation).
//
// Every function below follows the paper's text step by step:
//   * problem statement: discrete dynamics x_{t+1} = F(x_t, v_t), v_t ~ N(u_t, Sigma)
//     (Section II, Eq. Dynamics and the noise model below it);
//   * Algorithm 1 (Sampling Based MPC): sample E^k, roll out, accumulate
//     S_k += c(x) + gamma u^T Sigma^-1 (.), weights, U <- U + SGF * sum_k w_k E^k,
//     send u_0, shift, u_{T-1} <- Initialize;
//   * Algorithm 2 (Information Theoretic Weight Computation): rho = min S,
//     eta~ = sum exp(-(S-rho)/lambda), w = exp(-(S-rho)/lambda)/eta~;
//   * Section III-D-2 (decoupled control cost gamma), III-D-3 (clamp g inside the
//     dynamics), III-D-4 (Savitzky-Golay smoothing);
//   * Section VI-B (kinematic/dynamic state split, explicit Euler, 6-32-32-4 tanh
//     network) and VI-C (track, speed and stabilising costs).
// Readings of the paper where it is silent or ambiguous are listed in the
// design notes; the ones that change arithmetic are repeated at the point of use.
//
// Noise: the paper only says "sample epsilon ~ N(0, Sigma)".  This project fixes
// one counter-based generator so that the oracle and the GPU draw identical
// perturbations: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11) with counter (t, k, iter, instance) and key
// (seed_lo, seed_hi), then the Box-Muller transform (Box & Muller 1958) with an
// FP32 log and sin/cos defined below from textbook series.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

extern "C" {

typedef struct {
  int32_t K, T, hidden;
  float dt, lambda, gamma;
  float sigma2[2];          // covariance diagonal (variances)
  float u_lo[2], u_hi[2];   // clamp g
  int32_t sg_window, sg_order;
  float w_map, w_speed, w_slip, v_des;
  float crash_cost, crash_decay, map_thresh, slip_cost, slip_thresh;
  int32_t H, W;
  float origin_x, origin_y, resolution;
  const float* map;         // [H][W]
  const float* params;      // packed W1,b1,W2,b2,W3,b3 (row-major [out][in])
  uint64_t seed;
  uint32_t instance;
  float explore;            // exploration fraction alpha of Algorithm 1 (0 = none)
  int32_t weighting;        // ORC_WEIGHTS_IT (Algorithm 2) or ORC_WEIGHTS_CEM (Algorithm 3)
  float elite;              // Algorithm 3's eliteness threshold delta, in [0, 1)
  int32_t model;            // ORC_MODEL_NET (params = network) or ORC_MODEL_BASIS (params = Theta[25][4])
  int32_t nthreads;
} orc_problem;

enum { ORC_OK = 0, ORC_E_INVAL = 1, ORC_E_NONFINITE = 5 };
enum { ORC_WEIGHTS_IT = 0, ORC_WEIGHTS_CEM = 1 };
enum { ORC_MODEL_NET = 0, ORC_MODEL_BASIS = 1 };
enum { ORC_NBASIS = 25 };

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al. 2011): 10 rounds of the 4x32 Philox S-box with
// multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 /
// 0xBB67AE85.  One round maps (c0,c1,c2,c3) with key (k0,k1) to
//   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)).
// ---------------------------------------------------------------------------
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;   // the key bump after the last round is unused
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

// ---------------------------------------------------------------------------
// Noise transform (project definition, FP32, explicit fma, no contraction).
// Uniforms: u = (2*(w >> 9) + 1) * 2^-24, exact in FP32 and strictly inside (0,1).
// ---------------------------------------------------------------------------

// ln(u) for u built from word w.  u = n * 2^-24 with odd n < 2^24; n = 2^e * f,
// f in [1,2) (halved once more if f >= sqrt 2), ln f = 2 atanh(s), s = (f-1)/(f+1),
// atanh(s) = s + s^3/3 + ... + s^11/11, evaluated as s + (s*z)*P(z), z = s^2,
// P(z) = 1/3 + z/5 + z^2/7 + z^3/9 + z^4/11 (coefficients rounded to FP32).
float noise_log(uint32_t w) {
  const uint32_t n = 2u * (w >> 9) + 1u;
  int e = 0;
  while ((n >> (e + 1)) != 0u) ++e;                       // floor(log2 n)
  float f = std::ldexp((float)n, -e);                     // exact, in [1,2)
  if (f >= (float)std::sqrt(2.0)) { f = f * 0.5f; e += 1; }
  const float c3 = (float)(1.0 / 3.0), c5 = (float)(1.0 / 5.0), c7 = (float)(1.0 / 7.0);
  const float c9 = (float)(1.0 / 9.0), c11 = (float)(1.0 / 11.0);
  const float s = (f - 1.0f) / (f + 1.0f);
  const float z = s * s;
  float p = c11;
  p = std::fma(p, z, c9);
  p = std::fma(p, z, c7);
  p = std::fma(p, z, c5);
  p = std::fma(p, z, c3);
  const float at = std::fma(s * z, p, s);
  return std::fma((float)(e - 24), (float)std::log(2.0), 2.0f * at);
}

// cos(2 pi u), sin(2 pi u) for u built from word w.  2 pi u = (pi/2)(q + r) with
// q the nearest quadrant (integer arithmetic on n) and r in (-1/2, 1/2) exact;
// sin((pi/2) r) and cos((pi/2) r) from their Taylor series to r^11 and r^12 with
// coefficients (-1)^j (pi/2)^n / n! rounded to FP32, Horner in r^2.
void noise_sincos(uint32_t w, float* cs_out, float* sn_out) {
  const uint32_t n = 2u * (w >> 9) + 1u;
  const uint32_t q = (n + (1u << 21)) >> 22;                 // 0..4
  const int32_t rr = (int32_t)n - (int32_t)(q << 22);        // |rr| < 2^21
  const float r = std::ldexp((float)rr, -22);
  double fact[13];
  fact[0] = 1.0;
  for (int i = 1; i <= 12; ++i) fact[i] = fact[i - 1] * i;
  const double hp = std::acos(-1.0) / 2.0;
  auto coef = [&](int m) {
    double v = std::pow(hp, m) / fact[m];
    return (float)(((m / 2) % 2) ? -v : v);
  };
  const float r2 = r * r;
  float ps = coef(11);
  ps = std::fma(ps, r2, coef(9));
  ps = std::fma(ps, r2, coef(7));
  ps = std::fma(ps, r2, coef(5));
  ps = std::fma(ps, r2, coef(3));
  ps = std::fma(ps, r2, coef(1));
  const float sn = r * ps;
  float pc = coef(12);
  pc = std::fma(pc, r2, coef(10));
  pc = std::fma(pc, r2, coef(8));
  pc = std::fma(pc, r2, coef(6));
  pc = std::fma(pc, r2, coef(4));
  pc = std::fma(pc, r2, coef(2));
  const float cs = std::fma(pc, r2, 1.0f);
  switch (q & 3u) {
    case 0: *cs_out = cs;  *sn_out = sn;  break;
    case 1: *cs_out = -sn; *sn_out = cs;  break;
    case 2: *cs_out = -cs; *sn_out = -sn; break;
    default: *cs_out = sn; *sn_out = -cs; break;
  }
}

// epsilon_{k,t} = sqrt(Sigma) * z, z ~ N(0, I_2) by Box-Muller on words (w0, w1)
// of the Philox block with counter (t, k, iter, instance) and key (seed_lo, seed_hi).
void noise_pair(uint32_t t, uint32_t k, uint32_t iter, uint32_t instance, uint64_t seed,
                const float sig[2], float out[2]) {
  const uint32_t ctr[4] = {t, k, iter, instance};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t wds[4];
  philox4x32_10(ctr, key, wds);
  const float L = noise_log(wds[0]);
  const float R = std::sqrt(-2.0f * L);
  float c, s;
  noise_sincos(wds[1], &c, &s);
  out[0] = sig[0] * (R * c);
  out[1] = sig[1] * (R * s);
}

// ---------------------------------------------------------------------------
// Problem, promoted to the working precision R.
// ---------------------------------------------------------------------------
template <class R>
struct Prob {
  int K, T, h;
  R dt, lambda, gamma;
  R sigma2[2], u_lo[2], u_hi[2];
  R w_map, w_speed, w_slip, v_des, crash_cost, map_thresh, slip_cost, slip_thresh;
  std::vector<R> decay;   // decay[t] = fl32(crash_decay^t), t = 0..T
  int H, W;
  R ox, oy, res;
  const float* map;
  int model;
  std::vector<R> W1, b1, W2, b2, W3, b3;
  std::vector<R> theta;   // basis-function model: Theta[i][o], row-major [25][4]
  double explore;   // alpha of Algorithm 1, exactly as given (float widened)

  // Algorithm 1 draws sample k (counted from 0) around the nominal controls when
  // k < (1 - alpha) K and around zero otherwise (the exploration samples of the
  // disturbance discussion in Section IV).  The comparison is made in FP64.
  bool exploration(int k) const { return !((double)k < (1.0 - explore) * (double)K); }
};

template <class R>
void load_params(Prob<R>& P, const float* pf, const double* pd) {
  const int h = P.h;
  auto take = [&](std::vector<R>& v, size_t n, size_t& off) {
    v.resize(n);
    for (size_t i = 0; i < n; ++i) v[i] = pd ? (R)pd[off + i] : (R)pf[off + i];
    off += n;
  };
  size_t off = 0;
  take(P.W1, (size_t)h * 6, off);
  take(P.b1, (size_t)h, off);
  take(P.W2, (size_t)h * h, off);
  take(P.b2, (size_t)h, off);
  take(P.W3, (size_t)4 * h, off);
  take(P.b3, 4, off);
}

template <class R>
Prob<R> make_prob(const orc_problem* p, const double* params_override = nullptr) {
  Prob<R> P;
  P.K = p->K; P.T = p->T; P.h = p->hidden;
  P.dt = (R)p->dt; P.lambda = (R)p->lambda; P.gamma = (R)p->gamma;
  for (int i = 0; i < 2; ++i) {
    P.sigma2[i] = (R)p->sigma2[i]; P.u_lo[i] = (R)p->u_lo[i]; P.u_hi[i] = (R)p->u_hi[i];
  }
  P.w_map = (R)p->w_map; P.w_speed = (R)p->w_speed; P.w_slip = (R)p->w_slip; P.v_des = (R)p->v_des;
  P.crash_cost = (R)p->crash_cost; P.map_thresh = (R)p->map_thresh;
  P.slip_cost = (R)p->slip_cost; P.slip_thresh = (R)p->slip_thresh;
  P.decay.resize(P.T + 1);
  for (int t = 0; t <= P.T; ++t) P.decay[t] = (R)(float)std::pow((double)p->crash_decay, (double)t);
  P.H = p->H; P.W = p->W;
  P.ox = (R)p->origin_x; P.oy = (R)p->origin_y; P.res = (R)p->resolution;
  P.map = p->map;
  P.explore = (double)p->explore;
  P.model = p->model;
  if (P.model == ORC_MODEL_BASIS) {
    P.theta.resize(ORC_NBASIS * 4);
    for (int i = 0; i < ORC_NBASIS * 4; ++i)
      P.theta[i] = params_override ? (R)params_override[i] : (R)p->params[i];
  } else {
    load_params(P, p->params, params_override);
  }
  return P;
}

template <class R> R my_tanh(R a) { return std::tanh(a); }

// The dynamics network f(x_d, v): 6 -> h -> h -> 4, tanh, tanh, linear
// (Section VI-B-2; 1412 parameters at h = 32).  Keeps the hidden activations
// for the adjoint when h1/h2 are given.
template <class R>
void mlp_forward(const Prob<R>& P, const R in[6], R out[4], R* h1, R* h2) {
  const int h = P.h;
  for (int i = 0; i < h; ++i) {
    R a = P.b1[i];
    for (int j = 0; j < 6; ++j) a += P.W1[i * 6 + j] * in[j];
    h1[i] = my_tanh(a);
  }
  for (int i = 0; i < h; ++i) {
    R a = P.b2[i];
    for (int j = 0; j < h; ++j) a += P.W2[i * h + j] * h1[j];
    h2[i] = my_tanh(a);
  }
  for (int o = 0; o < 4; ++o) {
    R a = P.b3[o];
    for (int j = 0; j < h; ++j) a += P.W3[o * h + j] * h2[j];
    out[o] = a;
  }
}

// Cost map h(p_x, p_y): bilinear interpolation of the grid, cell (i, j) at world
// (ox + j*res, oy + i*res), indices clamped to the map edge.  (The paper reads a
// CUDA texture with hardware interpolation, Section VI-C; this is the plain
// FP bilinear it stands for.)  Optional gradient with respect to (p_x, p_y).
template <class R>
R costmap(const Prob<R>& P, R px, R py, R* dhdx = nullptr, R* dhdy = nullptr) {
  if (!std::isfinite((double)px) || !std::isfinite((double)py)) {
    if (dhdx) { *dhdx = 0; *dhdy = 0; }
    return std::numeric_limits<R>::quiet_NaN();
  }
  R gx = (px - P.ox) / P.res;
  R gy = (py - P.oy) / P.res;
  gx = std::min(std::max(gx, (R)-1), (R)P.W);
  gy = std::min(std::max(gy, (R)-1), (R)P.H);
  const long j0 = (long)std::floor(gx), i0 = (long)std::floor(gy);
  const R fx = gx - (R)j0, fy = gy - (R)i0;
  auto m = [&](long i, long j) {
    i = std::min(std::max(i, 0L), (long)P.H - 1);
    j = std::min(std::max(j, 0L), (long)P.W - 1);
    return (R)P.map[(size_t)i * P.W + j];
  };
  const R m00 = m(i0, j0), m01 = m(i0, j0 + 1), m10 = m(i0 + 1, j0), m11 = m(i0 + 1, j0 + 1);
  if (dhdx) {
    *dhdx = ((1 - fy) * (m01 - m00) + fy * (m11 - m10)) / P.res;
    *dhdy = ((1 - fx) * (m10 - m00) + fx * (m11 - m01)) / P.res;
  }
  return (1 - fy) * ((1 - fx) * m00 + fx * m01) + fy * ((1 - fx) * m10 + fx * m11);
}

// State cost c(x) at step index t (Section VI-C):
//   w_map*(h + crash_cost*decay^t*[h > map_thresh])-style track term, written with
//   the impulse weight as its own parameter, + w_speed*(v_x - v_des)^2
//   + w_slip*zeta^2 + slip_cost*[|zeta| > slip_thresh], zeta = -atan2(v_y, |v_x|).
template <class R>
R state_cost(const Prob<R>& P, const R x[7], int t, R* grad = nullptr) {
  R dhdx = 0, dhdy = 0;
  const R h = costmap(P, x[0], x[1], grad ? &dhdx : nullptr, grad ? &dhdy : nullptr);
  R c = P.w_map * h;
  if (h > P.map_thresh) c += P.crash_cost * P.decay[t];
  const R dv = x[4] - P.v_des;
  c += P.w_speed * dv * dv;
  const R zeta = -std::atan2(x[5], std::fabs(x[4]));
  c += P.w_slip * zeta * zeta;
  if (std::fabs(zeta) > P.slip_thresh) c += P.slip_cost;
  if (grad) {
    for (int i = 0; i < 7; ++i) grad[i] = 0;
    grad[0] = P.w_map * dhdx;
    grad[1] = P.w_map * dhdy;
    grad[4] = 2 * P.w_speed * dv;
    const R den = x[4] * x[4] + x[5] * x[5];
    if (den > 0) {
      const R sgn = x[4] > 0 ? (R)1 : (x[4] < 0 ? (R)-1 : (R)0);
      grad[4] += 2 * P.w_slip * zeta * (x[5] * sgn / den);
      grad[5] += 2 * P.w_slip * zeta * (-std::fabs(x[4]) / den);
    }
  }
  return c;
}

template <class R> R clampv(R v, R lo, R hi) { return std::min(std::max(v, lo), hi); }

// The 25 basis functions of the basis-function model (appendix), written as printed.
// The appendix uses the bicycle-model names: r for the heading (yaw) rate and theta for
// the roll angle; in this state layout those are x_d[3] (theta-dot) and x_d[0] (r).
// u_delta = steering g(v)_1, u_F = throttle g(v)_2.
template <class R>
void basis_functions(const R xd[4], R u_delta, R u_F, R phi[ORC_NBASIS]) {
  const R roll = xd[0], vx = xd[1], vy = xd[2], yaw_rate = xd[3];
  const bool moving = vx > (R)0.1;
  const R alpha_f = moving ? std::atan(vy / vx + (R)0.45 * yaw_rate / vx - u_delta) : -u_delta;
  const R alpha_r = moving ? std::atan(vy / vx - (R)0.35 * yaw_rate / vx) : (R)0;
  const R tf = std::tan(alpha_f), tr = std::tan(alpha_r);
  const R sd = std::sin(u_delta);
  phi[0] = u_F;
  phi[1] = vx / 10;
  phi[2] = sd * tf / 1200;
  phi[3] = sd * tf * std::fabs(tf) / (1200.0 * 1200.0);
  phi[4] = sd * tf * tf * tf / (1200.0 * 1200.0 * 1200.0);
  phi[5] = yaw_rate * vy / 25;
  phi[6] = yaw_rate / 10;
  phi[7] = vy / 10;
  phi[8] = sd;
  phi[9] = moving ? (vy / vx) / 40 : (R)0;
  phi[10] = tf / 1400;
  phi[11] = tf * std::fabs(tf) / (1400.0 * 1400.0);
  phi[12] = tf * tf * tf / (1400.0 * 1400.0 * 1400.0);
  phi[13] = tr / 40;
  phi[14] = tr * std::fabs(tr) / (40.0 * 40.0);
  phi[15] = tr * tr * tr / (40.0 * 40.0 * 40.0);
  phi[16] = yaw_rate * vx / 50;
  phi[17] = roll;
  phi[18] = roll * yaw_rate;
  phi[19] = roll * vx / 3;
  phi[20] = roll * vx * yaw_rate / 5;
  phi[21] = vx * vx / 100;
  phi[22] = vx * vx * vx / 1000;
  phi[23] = u_F * u_F;
  phi[24] = u_F * u_F * u_F;
}

// f(x_d, v) = Theta^T phi(x_d, v) (Section VI-B-1).
template <class R>
void basis_forward(const Prob<R>& P, const R in[6], R out[4]) {
  R phi[ORC_NBASIS];
  basis_functions(in, in[4], in[5], phi);
  for (int o = 0; o < 4; ++o) {
    R a = 0;
    for (int i = 0; i < ORC_NBASIS; ++i) a += P.theta[i * 4 + o] * phi[i];
    out[o] = a;
  }
}

// One step of the full equations of motion (Section VI-B): kinematic states by
// explicit Euler with the pre-step state, dynamic states x_d += f(x_d, v) dt.
template <class R>
void dynamics_step(const Prob<R>& P, const R x[7], const R vc[2], R xn[7], R* h1, R* h2) {
  const R in[6] = {x[3], x[4], x[5], x[6], vc[0], vc[1]};
  R f[4];
  if (P.model == ORC_MODEL_BASIS) basis_forward(P, in, f);
  else mlp_forward(P, in, f, h1, h2);
  const R c = std::cos(x[2]), s = std::sin(x[2]);
  xn[0] = x[0] + P.dt * (c * x[4] - s * x[5]);
  xn[1] = x[1] + P.dt * (s * x[4] + c * x[5]);
  xn[2] = x[2] + P.dt * x[6];
  for (int i = 0; i < 4; ++i) xn[3 + i] = x[3 + i] + P.dt * f[i];
}

// Algorithm 1 inner loop for sample k.  The control applied is
//   v_t = u_t + eps_t  (importance sample)   or   v_t = eps_t  (exploration sample),
// the state advances as x <- F(x, g(v_t)), and the running cost is
//   S += c(x, t+1) + gamma * sum_i u_{t,i} delta_{t,i} / Sigma_ii,   delta_t = v_t - u_t.
// This is the paper's gamma u^T Sigma^-1 v written with v - u in place of v: the two
// differ by gamma * sum_t u_t^T Sigma^-1 u_t, which is the same for every sample, so
// weights and updates are unchanged.  For importance samples delta_t is eps_t
// itself (no rounding).  Non-finite state or cost gives S = +inf.
template <class R>
R rollout_one(const Prob<R>& P, const float* x0, const float* U, const float* eps_k,
              bool zero_mean, R* traj) {
  std::vector<R> h1(P.h), h2(P.h);
  R x[7];
  for (int i = 0; i < 7; ++i) x[i] = (R)x0[i];
  if (traj) for (int i = 0; i < 7; ++i) traj[i] = x[i];
  R S = 0;
  bool ok = true;
  for (int t = 0; t < P.T; ++t) {
    const R u[2] = {(R)U[2 * t], (R)U[2 * t + 1]};
    const R e[2] = {(R)eps_k[2 * t], (R)eps_k[2 * t + 1]};
    R v[2], d[2];
    for (int i = 0; i < 2; ++i) {
      v[i] = zero_mean ? e[i] : u[i] + e[i];
      d[i] = zero_mean ? e[i] - u[i] : e[i];
    }
    const R vc[2] = {clampv(v[0], P.u_lo[0], P.u_hi[0]), clampv(v[1], P.u_lo[1], P.u_hi[1])};
    R xn[7];
    dynamics_step(P, x, vc, xn, h1.data(), h2.data());
    for (int i = 0; i < 7; ++i) { x[i] = xn[i]; ok = ok && std::isfinite((double)x[i]); }
    if (traj) for (int i = 0; i < 7; ++i) traj[(size_t)(t + 1) * 7 + i] = x[i];
    S += state_cost(P, x, t + 1) +
         P.gamma * (u[0] * d[0] / P.sigma2[0] + u[1] * d[1] / P.sigma2[1]);
  }
  if (!ok || !std::isfinite((double)S)) S = std::numeric_limits<R>::infinity();
  return S;
}

template <class F>
void parallel_for(int n, int nthreads, F fn) {
  nthreads = std::max(1, std::min(nthreads, n));
  if (nthreads == 1) { for (int i = 0; i < n; ++i) fn(i); return; }
  std::vector<std::thread> th;
  for (int w = 0; w < nthreads; ++w) {
    th.emplace_back([=, &fn]() { for (int i = w; i < n; i += nthreads) fn(i); });
  }
  for (auto& t : th) t.join();
}

template <class R>
void rollout_all(const Prob<R>& P, int nthreads, const float* x0, const float* U, const float* eps,
                 R* S, R* traj) {
  parallel_for(P.K, nthreads, [&](int k) {
    S[k] = rollout_one(P, x0, U, eps + (size_t)k * P.T * 2, P.exploration(k),
                       traj ? traj + (size_t)k * (P.T + 1) * 7 : nullptr);
  });
}

void noise_all(const orc_problem* p, uint32_t iter, float* eps) {
  const float sig[2] = {std::sqrt(p->sigma2[0]), std::sqrt(p->sigma2[1])};
  for (int k = 0; k < p->K; ++k)
    for (int t = 0; t < p->T; ++t)
      noise_pair((uint32_t)t, (uint32_t)k, iter, p->instance, p->seed, sig,
                 eps + ((size_t)k * p->T + t) * 2);
}

// Algorithm 2: rho = min_k S_k (over finite costs), eta~ = sum_k exp(-(S_k-rho)/lambda),
// w_k = exp(-(S_k-rho)/lambda)/eta~ (Section III-D-1 shift).  Non-finite S_k get
// weight 0; if no cost is finite the status is NONFINITE.
int weights(int K, const double* S, double lambda, double* w, double* rho_out, double* eta_out) {
  double rho = std::numeric_limits<double>::infinity();
  for (int k = 0; k < K; ++k) if (std::isfinite(S[k]) && S[k] < rho) rho = S[k];
  if (!std::isfinite(rho)) {
    for (int k = 0; k < K; ++k) w[k] = 0;
    if (rho_out) *rho_out = rho;
    if (eta_out) *eta_out = 0;
    return ORC_E_NONFINITE;
  }
  double eta = 0;
  for (int k = 0; k < K; ++k) {
    w[k] = std::isfinite(S[k]) ? std::exp(-(S[k] - rho) / lambda) : 0.0;
    eta += w[k];
  }
  for (int k = 0; k < K; ++k) w[k] /= eta;
  if (rho_out) *rho_out = rho;
  if (eta_out) *eta_out = eta;
  return ORC_OK;
}

// Algorithm 3 (cross-entropy weights).  zeta = round(K (1 - delta)), rounded half away
// from zero in FP64 from the FP32 delta.  The elite set is read as the zeta samples of
// lowest cost -- the unweighted average over the best samples that Section V describes,
// and the elite set of its enumerated procedure (cost <= the zeta-th cost); taken
// literally, the strict comparison with the zeta-th cost would keep zeta - 1 samples
// with weights summing to (zeta - 1)/zeta.  Samples are ordered by (S_k, k), so equal
// costs go to the lower index; non-finite costs are never elite.  With n finite costs
// the elite set is the first min(zeta, n) in that order and every elite sample weighs
// 1/|E|.  z_out = the largest elite cost, n_out = |E|.
int cem_zeta(int K, float delta) {
  return (int)std::round((double)K * (1.0 - (double)delta));
}

int weights_cem(int K, const double* S, int zeta, double* w, double* z_out, double* n_out) {
  std::vector<int> idx;
  for (int k = 0; k < K; ++k) if (std::isfinite(S[k])) idx.push_back(k);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return S[a] < S[b] || (S[a] == S[b] && a < b); });
  const int n = std::min<int>(zeta, (int)idx.size());
  for (int k = 0; k < K; ++k) w[k] = 0.0;
  if (n_out) *n_out = (double)n;
  if (n == 0) {
    if (z_out) *z_out = std::numeric_limits<double>::infinity();
    return ORC_E_NONFINITE;
  }
  for (int i = 0; i < n; ++i) w[idx[i]] = 1.0 / (double)n;
  if (z_out) *z_out = S[idx[n - 1]];
  return ORC_OK;
}

// Savitzky-Golay smoothing (Section III-D-4) as a [T][T] matrix: row t evaluates at
// t the least-squares polynomial of degree `order` through the `window` points
// centred on t, or through the first / last `window` points near the ends.
void sgf_matrix(int T, int window, int order, double* M) {
  std::fill(M, M + (size_t)T * T, 0.0);
  const int hw = window / 2;
  const int n = order + 1;
  for (int t = 0; t < T; ++t) {
    const int lo = std::min(std::max(t - hw, 0), T - window);
    // normal equations G y = e0, G = A^T A with A[r][p] = (lo + r - t)^p
    std::vector<double> G((size_t)n * n, 0.0), y(n, 0.0);
    for (int r = 0; r < window; ++r) {
      const double d = (double)(lo + r - t);
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) G[a * n + b] += std::pow(d, a) * std::pow(d, b);
    }
    y[0] = 1.0;
    // Gaussian elimination with partial pivoting
    for (int c = 0; c < n; ++c) {
      int piv = c;
      for (int r = c + 1; r < n; ++r) if (std::fabs(G[r * n + c]) > std::fabs(G[piv * n + c])) piv = r;
      if (piv != c) {
        for (int b = 0; b < n; ++b) std::swap(G[c * n + b], G[piv * n + b]);
        std::swap(y[c], y[piv]);
      }
      for (int r = c + 1; r < n; ++r) {
        const double f = G[r * n + c] / G[c * n + c];
        for (int b = c; b < n; ++b) G[r * n + b] -= f * G[c * n + b];
        y[r] -= f * y[c];
      }
    }
    for (int c = n - 1; c >= 0; --c) {
      double s = y[c];
      for (int b = c + 1; b < n; ++b) s -= G[c * n + b] * y[b];
      y[c] = s / G[c * n + c];
    }
    for (int r = 0; r < window; ++r) {
      const double d = (double)(lo + r - t);
      double cr = 0;
      for (int a = 0; a < n; ++a) cr += y[a] * std::pow(d, a);
      M[(size_t)t * T + lo + r] = cr;
    }
  }
}

bool valid_problem(const orc_problem* p) {
  if (!p || p->K <= 0 || p->T <= 0) return false;
  if (p->model != ORC_MODEL_NET && p->model != ORC_MODEL_BASIS) return false;
  if (p->model == ORC_MODEL_NET && p->hidden <= 0) return false;
  if (!(p->sigma2[0] > 0 && p->sigma2[1] > 0 && p->lambda > 0)) return false;
  if (p->sg_window < 1 || p->sg_window % 2 == 0 || p->sg_window > p->T) return false;
  if (p->sg_order < 0 || p->sg_order >= p->sg_window) return false;
  if (!p->map || !p->params || p->H <= 0 || p->W <= 0 || !(p->resolution > 0)) return false;
  if (!(p->explore >= 0.0f && p->explore <= 1.0f)) return false;
  if (p->weighting != ORC_WEIGHTS_IT && p->weighting != ORC_WEIGHTS_CEM) return false;
  if (p->weighting == ORC_WEIGHTS_CEM &&
      !(p->elite >= 0.0f && p->elite < 1.0f && cem_zeta(p->K, p->elite) >= 1)) return false;
  return true;
}

}  // namespace

extern "C" {

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox4x32_10(ctr, key, out);
}

float orc_noise_log(uint32_t w) { return noise_log(w); }

void orc_noise_sincos(uint32_t w, float* c, float* s) { noise_sincos(w, c, s); }

void orc_noise(const orc_problem* p, uint32_t iter, float* eps) { noise_all(p, iter, eps); }

int orc_rollout_f64(const orc_problem* p, const float* x0, const float* U, const float* eps,
                    double* S, double* traj) {
  if (!valid_problem(p)) return ORC_E_INVAL;
  Prob<double> P = make_prob<double>(p);
  rollout_all(P, p->nthreads, x0, U, eps, S, traj);
  return ORC_OK;
}

int orc_rollout_f32(const orc_problem* p, const float* x0, const float* U, const float* eps,
                    float* S, float* traj) {
  if (!valid_problem(p)) return ORC_E_INVAL;
  Prob<float> P = make_prob<float>(p);
  rollout_all(P, p->nthreads, x0, U, eps, S, traj);
  return ORC_OK;
}

int orc_weights(int K, const double* S, double lambda, double* w, double* rho, double* eta) {
  return weights(K, S, lambda, w, rho, eta);
}

int orc_cem_zeta(int K, float delta) { return cem_zeta(K, delta); }

int orc_weights_cem(int K, const double* S, int zeta, double* w, double* z, double* n) {
  if (K < 1 || zeta < 1) return ORC_E_INVAL;
  return weights_cem(K, S, zeta, w, z, n);
}

void orc_sgf_matrix(int T, int window, int order, double* M) { sgf_matrix(T, window, order, M); }

// One iteration of Algorithm 1 (without the shift): noise, rollouts, weights
// (Algorithm 2, or Algorithm 3 for the cross-entropy variant),
// Delta_t = sum_k w_k delta_{k,t}, U_out = U + SGF * Delta, where delta_{k,t} =
// v_{k,t} - u_t is eps_{k,t} for importance samples and eps_{k,t} - u_t for
// exploration samples.  (Algorithm 1 writes the sum with E^k for every sample; with
// exploration samples that is not the optimal-control update of Eq. IT-Controls,
// u* = sum_k w_k v_k = u + sum_k w_k (v_k - u), which is what is computed here.)
// Outputs in FP64.
// eps_in (nullable) overrides the generated noise.  rho_eta_out = {rho, eta~}.
int orc_iterate(const orc_problem* p, const float* x0, const float* U, uint32_t iter,
                const float* eps_in, double* U_out, double* S_out, double* w_out,
                double* delta_out, double* rho_eta_out) {
  if (!valid_problem(p)) return ORC_E_INVAL;
  const int K = p->K, T = p->T;
  std::vector<float> eps_gen;
  const float* eps = eps_in;
  if (!eps) { eps_gen.resize((size_t)K * T * 2); noise_all(p, iter, eps_gen.data()); eps = eps_gen.data(); }
  Prob<double> P = make_prob<double>(p);
  std::vector<double> S(K), w(K), delta((size_t)T * 2, 0.0), M((size_t)T * T);
  rollout_all(P, p->nthreads, x0, U, eps, S.data(), (double*)nullptr);
  double rho = 0, eta = 0;
  const int st = p->weighting == ORC_WEIGHTS_CEM
                     ? weights_cem(K, S.data(), cem_zeta(K, p->elite), w.data(), &rho, &eta)
                     : weights(K, S.data(), (double)p->lambda, w.data(), &rho, &eta);
  if (S_out) std::copy(S.begin(), S.end(), S_out);
  if (w_out) std::copy(w.begin(), w.end(), w_out);
  if (rho_eta_out) { rho_eta_out[0] = rho; rho_eta_out[1] = eta; }
  for (int i = 0; i < 2 * T; ++i) U_out[i] = (double)U[i];
  if (st != ORC_OK) { if (delta_out) std::fill(delta_out, delta_out + 2 * T, 0.0); return st; }
  for (int k = 0; k < K; ++k) {
    const bool zero_mean = P.exploration(k);
    for (int i = 0; i < 2 * T; ++i) {
      const double e = (double)eps[(size_t)k * T * 2 + i];
      delta[i] += w[k] * (zero_mean ? e - (double)U[i] : e);
    }
  }
  if (delta_out) std::copy(delta.begin(), delta.end(), delta_out);
  sgf_matrix(T, p->sg_window, p->sg_order, M.data());
  for (int t = 0; t < T; ++t)
    for (int c = 0; c < 2; ++c) {
      double s = 0;
      for (int j = 0; j < T; ++j) s += M[(size_t)t * T + j] * delta[2 * j + c];
      U_out[2 * t + c] += s;
    }
  return ORC_OK;
}

// Algorithm 1's last block: u_0 goes to the actuators, u_{t-1} <- u_t, u_{T-1} <- (0,0)
// (Table 2 "Initialize").
void orc_shift(int T, const double* U, double* U_out, double* u0) {
  u0[0] = U[0]; u0[1] = U[1];
  for (int t = 0; t + 1 < T; ++t) { U_out[2 * t] = U[2 * t + 2]; U_out[2 * t + 1] = U[2 * t + 3]; }
  U_out[2 * (T - 1)] = 0.0; U_out[2 * (T - 1) + 1] = 0.0;
}

// Noise-free plant step x_out = F(x, g(u)) with the problem's network (FP64).
void orc_plant_step(const orc_problem* p, const double* x, const double* u, double* x_out) {
  Prob<double> P = make_prob<double>(p);
  std::vector<double> h1(P.h), h2(P.h);
  const double vc[2] = {clampv(u[0], P.u_lo[0], P.u_hi[0]), clampv(u[1], P.u_lo[1], P.u_hi[1])};
  dynamics_step(P, x, vc, x_out, h1.data(), h2.data());
}

// Free-energy objective J = -lambda log((1/K) sum_k exp(-S_k/lambda))
//   = rho - lambda log(eta~/K)            (Eq. FreeEnergy with the Monte-Carlo
// estimate over the K samples of this iteration's noise), evaluated at FP64
// nominal controls U and FP64 network parameters (nullable: use the problem's).
// Defined for importance samples, Algorithm 2's weights and the network model only
// (otherwise INVAL).
int orc_objective(const orc_problem* p, const float* x0, const double* U, const double* params,
                  uint32_t iter, double* J, double* S_out) {
  if (!valid_problem(p)) return ORC_E_INVAL;
  // defined for importance samples, the information-theoretic weights and the network
  if (p->explore != 0.0f || p->weighting != ORC_WEIGHTS_IT || p->model != ORC_MODEL_NET) return ORC_E_INVAL;
  const int K = p->K, T = p->T;
  std::vector<float> eps((size_t)K * T * 2);
  noise_all(p, iter, eps.data());
  Prob<double> P = make_prob<double>(p, params);
  std::vector<double> S(K), w(K);
  parallel_for(K, p->nthreads, [&](int k) {
    std::vector<double> h1(P.h), h2(P.h);
    double x[7];
    for (int i = 0; i < 7; ++i) x[i] = (double)x0[i];
    double s = 0;
    bool ok = true;
    const float* ek = eps.data() + (size_t)k * T * 2;
    for (int t = 0; t < T; ++t) {
      const double u[2] = {U[2 * t], U[2 * t + 1]};
      const double e[2] = {(double)ek[2 * t], (double)ek[2 * t + 1]};
      const double vc[2] = {clampv(u[0] + e[0], P.u_lo[0], P.u_hi[0]),
                            clampv(u[1] + e[1], P.u_lo[1], P.u_hi[1])};
      double xn[7];
      dynamics_step(P, x, vc, xn, h1.data(), h2.data());
      for (int i = 0; i < 7; ++i) { x[i] = xn[i]; ok = ok && std::isfinite(x[i]); }
      s += state_cost(P, x, t + 1) + P.gamma * (u[0] * e[0] / P.sigma2[0] + u[1] * e[1] / P.sigma2[1]);
    }
    S[k] = (ok && std::isfinite(s)) ? s : std::numeric_limits<double>::infinity();
  });
  double rho = 0, eta = 0;
  const int st = weights(K, S.data(), (double)p->lambda, w.data(), &rho, &eta);
  if (S_out) std::copy(S.begin(), S.end(), S_out);
  if (st != ORC_OK) return st;
  *J = rho - (double)p->lambda * std::log(eta / (double)K);
  return ORC_OK;
}

// Gradient of J with respect to U ([T][2]) and the packed network parameters, by
// reverse-mode over the stored trajectory of every sample (FP64, no checkpointing):
//   dJ/dS_k = w_k;  p_{t+1} <- p_{t+1} + grad c(x_{t+1});  dS/du_t = g'(v_t) (dF/dv)^T p_{t+1}
//   + gamma eps_t / Sigma;  dS/dtheta += (dF/dtheta)^T p_{t+1};  p_t = (dF/dx_t)^T p_{t+1}.
// g' = 1 strictly inside (u_lo, u_hi), 0 otherwise; impulse indicators contribute 0.
int orc_objective_grad(const orc_problem* p, const float* x0, const double* U, const double* params,
                       uint32_t iter, double* J, double* dJdU, double* dJdtheta) {
  if (!valid_problem(p)) return ORC_E_INVAL;
  if (p->explore != 0.0f || p->weighting != ORC_WEIGHTS_IT || p->model != ORC_MODEL_NET) return ORC_E_INVAL;
  const int K = p->K, T = p->T, h = p->hidden;
  std::vector<float> eps((size_t)K * T * 2);
  noise_all(p, iter, eps.data());
  Prob<double> P = make_prob<double>(p, params);
  const size_t NP = (size_t)6 * h + h + (size_t)h * h + h + 4 * (size_t)h + 4;
  std::vector<double> S(K), w(K);
  std::vector<double> gU((size_t)K * T * 2), gTh((size_t)K * NP);
  parallel_for(K, p->nthreads, [&](int k) {
    const float* ek = eps.data() + (size_t)k * T * 2;
    std::vector<double> X((size_t)(T + 1) * 7), H1((size_t)T * h), H2((size_t)T * h);
    std::vector<double> VC((size_t)T * 2), V((size_t)T * 2);
    for (int i = 0; i < 7; ++i) X[i] = (double)x0[i];
    double s = 0;
    bool ok = true;
    for (int t = 0; t < T; ++t) {
      const double u[2] = {U[2 * t], U[2 * t + 1]};
      const double e[2] = {(double)ek[2 * t], (double)ek[2 * t + 1]};
      V[2 * t] = u[0] + e[0]; V[2 * t + 1] = u[1] + e[1];
      VC[2 * t] = clampv(V[2 * t], P.u_lo[0], P.u_hi[0]);
      VC[2 * t + 1] = clampv(V[2 * t + 1], P.u_lo[1], P.u_hi[1]);
      dynamics_step(P, &X[(size_t)t * 7], &VC[2 * t], &X[(size_t)(t + 1) * 7], &H1[(size_t)t * h], &H2[(size_t)t * h]);
      for (int i = 0; i < 7; ++i) ok = ok && std::isfinite(X[(size_t)(t + 1) * 7 + i]);
      s += state_cost(P, &X[(size_t)(t + 1) * 7], t + 1) +
           P.gamma * (u[0] * e[0] / P.sigma2[0] + u[1] * e[1] / P.sigma2[1]);
    }
    S[k] = (ok && std::isfinite(s)) ? s : std::numeric_limits<double>::infinity();
    // adjoint sweep
    double* gu = &gU[(size_t)k * T * 2];
    double* gth = &gTh[(size_t)k * NP];
    std::fill(gth, gth + NP, 0.0);
    double* gW1 = gth;
    double* gb1 = gW1 + 6 * h;
    double* gW2 = gb1 + h;
    double* gb2 = gW2 + (size_t)h * h;
    double* gW3 = gb2 + h;
    double* gb3 = gW3 + 4 * h;
    double pa[7] = {0, 0, 0, 0, 0, 0, 0};
    std::vector<double> gh2(h), ga2(h), gh1(h), ga1(h);
    for (int t = T - 1; t >= 0; --t) {
      double gc[7];
      state_cost(P, &X[(size_t)(t + 1) * 7], t + 1, gc);
      for (int i = 0; i < 7; ++i) pa[i] += gc[i];
      const double* x = &X[(size_t)t * 7];
      const double* h1 = &H1[(size_t)t * h];
      const double* h2 = &H2[(size_t)t * h];
      const double in[6] = {x[3], x[4], x[5], x[6], VC[2 * t], VC[2 * t + 1]};
      // network backward with upstream dt * p[3:7]
      double ga3[4];
      for (int o = 0; o < 4; ++o) ga3[o] = P.dt * pa[3 + o];
      for (int o = 0; o < 4; ++o) {
        gb3[o] += ga3[o];
        for (int j = 0; j < h; ++j) gW3[o * h + j] += ga3[o] * h2[j];
      }
      for (int j = 0; j < h; ++j) {
        double g = 0;
        for (int o = 0; o < 4; ++o) g += P.W3[o * h + j] * ga3[o];
        gh2[j] = g;
        ga2[j] = g * (1 - h2[j] * h2[j]);
      }
      for (int i = 0; i < h; ++i) {
        gb2[i] += ga2[i];
        for (int j = 0; j < h; ++j) gW2[i * h + j] += ga2[i] * h1[j];
      }
      for (int j = 0; j < h; ++j) {
        double g = 0;
        for (int i = 0; i < h; ++i) g += P.W2[i * h + j] * ga2[i];
        gh1[j] = g;
        ga1[j] = g * (1 - h1[j] * h1[j]);
      }
      double gin[6] = {0, 0, 0, 0, 0, 0};
      for (int i = 0; i < h; ++i) {
        gb1[i] += ga1[i];
        for (int j = 0; j < 6; ++j) { gW1[i * 6 + j] += ga1[i] * in[j]; gin[j] += P.W1[i * 6 + j] * ga1[i]; }
      }
      // control gradient
      for (int c = 0; c < 2; ++c) {
        const double v = V[2 * t + c];
        const double gprime = (v > P.u_lo[c] && v < P.u_hi[c]) ? 1.0 : 0.0;
        gu[2 * t + c] = gprime * gin[4 + c] + P.gamma * (double)ek[2 * t + c] / P.sigma2[c];
      }
      // state adjoint p_t = (dF/dx_t)^T p_{t+1}
      const double c = std::cos(x[2]), sn = std::sin(x[2]);
      double np[7];
      np[0] = pa[0];
      np[1] = pa[1];
      np[2] = pa[2] + P.dt * (pa[0] * (-sn * x[4] - c * x[5]) + pa[1] * (c * x[4] - sn * x[5]));
      np[3] = pa[3] + gin[0];
      np[4] = pa[4] + P.dt * (pa[0] * c + pa[1] * sn) + gin[1];
      np[5] = pa[5] + P.dt * (-pa[0] * sn + pa[1] * c) + gin[2];
      np[6] = pa[6] + P.dt * pa[2] + gin[3];
      for (int i = 0; i < 7; ++i) pa[i] = np[i];
    }
  });
  double rho = 0, eta = 0;
  const int st = weights(K, S.data(), (double)p->lambda, w.data(), &rho, &eta);
  if (st != ORC_OK) return st;
  *J = rho - (double)p->lambda * std::log(eta / (double)K);
  std::fill(dJdU, dJdU + (size_t)T * 2, 0.0);
  std::fill(dJdtheta, dJdtheta + NP, 0.0);
  for (int k = 0; k < K; ++k) {
    if (w[k] == 0.0) continue;
    for (int i = 0; i < 2 * T; ++i) dJdU[i] += w[k] * gU[(size_t)k * T * 2 + i];
    for (size_t i = 0; i < NP; ++i) dJdtheta[i] += w[k] * gTh[(size_t)k * NP + i];
  }
  return ORC_OK;
}

// Per sample, the smallest distance over t = 1..T of the map value to map_thresh
// and of |zeta| to slip_thresh along the FP64 trajectory (and, with the basis-function
// model, of v_x to its 0.1 branch point over t = 0..T-1): samples that pass within a
// rounding error of such a threshold can legitimately take the other side of it.
int orc_threshold_margins(const orc_problem* p, const float* x0, const float* U, const float* eps,
                          double* margin) {
  if (!valid_problem(p)) return ORC_E_INVAL;
  Prob<double> P = make_prob<double>(p);
  const int T = P.T;
  parallel_for(P.K, p->nthreads, [&](int k) {
    std::vector<double> tr((size_t)(T + 1) * 7);
    rollout_one(P, x0, U, eps + (size_t)k * T * 2, P.exploration(k), tr.data());
    double m = std::numeric_limits<double>::infinity();
    // the basis-function model branches on v_x > 0.1 at the states entering each step
    if (P.model == ORC_MODEL_BASIS)
      for (int t = 0; t < T; ++t) m = std::min(m, std::fabs(tr[(size_t)t * 7 + 4] - 0.1));
    for (int t = 1; t <= T; ++t) {
      const double* x = &tr[(size_t)t * 7];
      const double h = costmap(P, x[0], x[1]);
      const double zeta = -std::atan2(x[5], std::fabs(x[4]));
      if (std::isfinite((double)P.map_thresh)) m = std::min(m, std::fabs(h - P.map_thresh));
      if (std::isfinite((double)P.slip_thresh)) m = std::min(m, std::fabs(std::fabs(zeta) - P.slip_thresh));
    }
    margin[k] = m;
  });
  return ORC_OK;
}

// The impulse terms of the state cost (Section VI-C) whose indicator the FP64 trajectory
// of a sample decides within `window` of its threshold: the crash term
// crash_cost * decay_t * [h > map_thresh] (kind 0) and the slip term
// slip_cost * [|zeta| > slip_thresh] (kind 1), at post-step states t = 1..T.  A
// computation whose trajectory differs from this one by rounding may take either side of
// such an indicator; every other indicator it must take as here.  The indicators do not
// feed back into the trajectory, so the costs such a computation may legitimately report
// are exactly S_ref - sum(on * value) + (any subset sum of the values).  Per sample k:
// n_out[k] = the number of such terms (all of them are counted; the first `cap` are
// listed in t_out / kind_out / value_out / on_out [k][cap], in t order, crash before slip).
int orc_threshold_events(const orc_problem* p, const float* x0, const float* U, const float* eps,
                         double window, int32_t cap, int32_t* n_out, int32_t* t_out, int32_t* kind_out,
                         double* value_out, int32_t* on_out) {
  if (!valid_problem(p) || cap < 0 || !(window >= 0)) return ORC_E_INVAL;
  Prob<double> P = make_prob<double>(p);
  const int T = P.T;
  parallel_for(P.K, p->nthreads, [&](int k) {
    std::vector<double> tr((size_t)(T + 1) * 7);
    rollout_one(P, x0, U, eps + (size_t)k * T * 2, P.exploration(k), tr.data());
    int n = 0;
    auto add = [&](int t, int kind, double value, bool on) {
      if (n < cap) {
        const size_t i = (size_t)k * cap + n;
        t_out[i] = t;
        kind_out[i] = kind;
        value_out[i] = value;
        on_out[i] = on ? 1 : 0;
      }
      ++n;
    };
    for (int t = 1; t <= T; ++t) {
      const double* x = &tr[(size_t)t * 7];
      const double h = costmap(P, x[0], x[1]);
      const double zeta = -std::atan2(x[5], std::fabs(x[4]));
      if (std::isfinite((double)P.map_thresh) && std::fabs(h - P.map_thresh) < window)
        add(t, 0, P.crash_cost * P.decay[t], h > P.map_thresh);
      if (std::isfinite((double)P.slip_thresh) && std::fabs(std::fabs(zeta) - P.slip_thresh) < window)
        add(t, 1, P.slip_cost, std::fabs(zeta) > P.slip_thresh);
    }
    n_out[k] = n;
  });
  return ORC_OK;
}

// Single-step pieces, exported so each can be pinned on its own.
int orc_mlp_forward(const orc_problem* p, const double* in, double* out) {
  if (!p || !p->params || p->hidden <= 0) return ORC_E_INVAL;
  Prob<double> P;
  P.h = p->hidden;
  load_params(P, p->params, nullptr);
  std::vector<double> h1(P.h), h2(P.h);
  mlp_forward(P, in, out, h1.data(), h2.data());
  return ORC_OK;
}

void orc_basis_phi(const double xd[4], const double u[2], double phi[ORC_NBASIS]) {
  basis_functions(xd, u[0], u[1], phi);
}

double orc_costmap(const orc_problem* p, double px, double py, double* grad2) {
  Prob<double> P = make_prob<double>(p);
  double gx = 0, gy = 0;
  const double h = costmap(P, px, py, &gx, &gy);
  if (grad2) { grad2[0] = gx; grad2[1] = gy; }
  return h;
}

double orc_state_cost(const orc_problem* p, const double* x, int t, double* grad7) {
  Prob<double> P = make_prob<double>(p);
  return state_cost(P, x, t, grad7);
}

// Linear-Gaussian toy with scalar state and control: x_{t+1} = a x_t + b v_t,
// c(x) = q x^2 on x_1..x_T, v_t = u_t + eps_t, eps_t ~ N(0, sigma2) from channel 0
// of the same noise contract, control cost gamma = lambda in the epsilon form, and
// the same weight computation (Algorithm 2) and update U <- U + sum_k w_k E^k.
// ctrl_scale multiplies the control-cost term; 1 is the method, 0 plants the
// mistake of dropping it (used only to show that the closed-form pin detects it).
int orc_toy_iterate(double a, double b, double q, float lambda, float sigma2, double x0, int T,
                    int K, const double* U, uint64_t seed, uint32_t iter, double ctrl_scale,
                    double* U_out) {
  if (K <= 0 || T <= 0 || !(lambda > 0) || !(sigma2 > 0)) return ORC_E_INVAL;
  const float sig[2] = {std::sqrt(sigma2), std::sqrt(sigma2)};
  std::vector<double> S(K), w(K), E((size_t)K * T);
  for (int k = 0; k < K; ++k) {
    double x = x0, s = 0;
    for (int t = 0; t < T; ++t) {
      float e2[2];
      noise_pair((uint32_t)t, (uint32_t)k, iter, 0u, seed, sig, e2);
      const double e = (double)e2[0];
      E[(size_t)k * T + t] = e;
      x = a * x + b * (U[t] + e);
      s += q * x * x + ctrl_scale * (double)lambda * U[t] * e / (double)sigma2;
    }
    S[k] = s;
  }
  const int st = weights(K, S.data(), (double)lambda, w.data(), nullptr, nullptr);
  for (int t = 0; t < T; ++t) U_out[t] = U[t];
  if (st != ORC_OK) return st;
  for (int k = 0; k < K; ++k)
    for (int t = 0; t < T; ++t) U_out[t] += w[k] * E[(size_t)k * T + t];
  return ORC_OK;
}

}  // extern "C"
