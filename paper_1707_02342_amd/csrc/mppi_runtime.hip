// Host runtime of libmppi.so: the C ABI declared in include/mppi.h.
//
// The context owns every device buffer, binds one HIP stream, validates every
// argument before anything is enqueued, and launches the rollout kernel (one
// of two schedules) per iteration; its last block forms the weights and updates U.
// No C++ exception escapes: every entry point catches and maps to a status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mppi.h"
#include "mppi_types.h"

namespace mppi {
hipError_t launch_lane(int precision, int hidden, dim3 grid, hipStream_t stream, const RolloutArgs& a);
template <int HID, int NQ, int MODEL> __global__ void rollout_wave_kernel(RolloutArgs);
size_t wave_smem_bytes(int T, int model);
template <int MODEL, bool MULTI> __global__ void rollout_wave_split_kernel(RolloutArgs);
size_t wave_split_smem_bytes(int T, int model);
constexpr int kWaveSplitBlockThreads = 512;   // 4 chain waves + 4 cost waves
constexpr int kWaveSplitMaxT = 128;
size_t wide_smem_bytes(int T);
template <int NQ> __global__ void rollout_wide_kernel(RolloutArgs);
template <int PREC, int HID> __global__ void rollout_quad_kernel(RolloutArgs);
__global__ void shift_kernel(float*, int, float*);
__global__ void merge_update_kernel(RolloutArgs, const float*, int);
template <int HID>
__global__ void plant_kernel(const float*, const float*, const float*, float*, float*, float, float,
                             float, float, float);
__global__ void noise_kernel(NoiseKey, int, int, float*);
__global__ void costmap_kernel(CostArgs, const float*, const float*, int, float*);
__global__ void adjoint_wave_kernel(AdjointArgs);
template <int NCOL, int HC> __global__ void cem_update_kernel(RolloutArgs);
constexpr int kCemBlockThreads = 1024;
__global__ void adjoint_reduce_partial_kernel(const float*, int, int, int, float*);
__global__ void adjoint_reduce_final_kernel(const float*, int, int, const float*, float, float, float*);
constexpr int kGradChunks = 16;   // row chunks of the first gradient reduction pass
size_t adjoint_smem_bytes(int T, int ckpt_every);
constexpr int kNP32Host = 1412;
constexpr int kLaneBlockHost = 256;
constexpr int kWaveSamplesPerBlock = 8;   // 4 waves x 2 samples of 32 lanes
constexpr int kWaveBlockThreads = 256;
constexpr int kWideSamplesPerBlock = 8;   // 8 waves x 1 sample of 64 lanes
constexpr int kWideBlockThreads = 512;
constexpr int kQuadSamplesPerBlock = 64;  // 4 waves x 16 samples of 4 lanes
constexpr int kQuadBlockThreads = 256;
}  // namespace mppi

using namespace mppi;

namespace {

thread_local std::string g_create_error;

constexpr int32_t kMaxK = 1 << 22;
// Automatic schedule: 32 lanes per sample while that still fits the chip in a few
// waves per SIMD (latency-bound regime), one lane per sample beyond.
constexpr int32_t kWaveAutoMaxK = 12288;   // AUTO: WAVE up to here, QUAD above
constexpr int kNumBasisHost = 25;          // basis functions of the basis-function model

struct PendingTiming {
  hipEvent_t e0, e1;
  int slot = 0;   // 0: the iteration's rollout launch, 1: the adjoint rollout kernel
};

}  // namespace

struct mppi_ctx {
  mppi_config cfg{};
  mppi_cost cost{};
  int device = 0;
  hipStream_t stream = nullptr;
  int hidden = 0;
  int model = kModelNet;     // kModelNet or kModelBasis (set by the last set_*dynamics call)
  size_t n_params = 0;       // floats in d_params
  bool have_map = false, have_dyn = false;
  int H = 0, W = 0;
  float ox = 0, oy = 0, res = 1;
  float* d_U = nullptr;
  float* d_map = nullptr;
  float* d_params = nullptr;
  float* d_decay = nullptr;
  float* d_S = nullptr;
  float* d_D = nullptr;      // Algorithm 3 only: [K][T][2] delta rows
  float* d_eps = nullptr;    // quad schedule: the noise of a launch's tiles [G][4][T][16][2]
  float* d_part = nullptr;
  float* d_part2 = nullptr;
  unsigned* d_cnt = nullptr;
  float* d_stats = nullptr;
  float* d_sg = nullptr;
  float* d_x = nullptr;      // [7] device-resident state for the receding loop
  float* d_u0 = nullptr;     // [2]
  int* d_status = nullptr;
  float* d_hist_u = nullptr;
  float* d_hist_x = nullptr;
  int hist_cap = 0;
  float* d_ckpt = nullptr;    // objective checkpoints [K][n_ckpt][8]
  float* d_gpart = nullptr;   // adjoint per-block partials
  float* d_gout = nullptr;    // reduced gradient [1412 + 2T]
  float* d_gred = nullptr;    // chunk sums of the gradient partials [16][1412 + 2T]
  unsigned* d_iter = nullptr; // the iteration counter (Philox counter word 3), advanced on the device
  unsigned* d_sync = nullptr; // signal words of multi-step receding launches ([kSyncWords(part_cap)])
  unsigned step_count = 0;    // steps of the multi-step launches enqueued so far (their signal base)
  int ckpt_cap = 0;           // n_ckpt the checkpoint buffer holds
  bool objective_ready = false;
  int obj_ckpt_every = 0;
  uint32_t obj_iter = 0;
  int part_cap = 0;          // partial rows allocated
  int ngrp_cap = 0;          // group rows allocated (arrival counters: ngrp_cap + 1)
  uint32_t iter = 0;
  int schedule = MPPI_SCHED_LANE;
  float sig[2] = {0, 0};
  std::string err;
  bool timing = false;
  std::vector<PendingTiming> pending;
  std::vector<hipEvent_t> event_pool;
  double t_ms[2] = {0, 0};
  std::vector<float> t_samples;   // per-launch kernel durations (ms) since timing was enabled
  int64_t t_cnt[2] = {0, 0};
};

namespace {

mppi_status fail(mppi_ctx* c, mppi_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf; else g_create_error = buf;
  return st;
}

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail((ctx), e_ == hipErrorOutOfMemory ? MPPI_E_NOMEM : MPPI_E_DEVICE, "%s: %s", \
                  #expr, hipGetErrorString(e_));                                             \
  } while (0)

bool finite(float v) { return std::isfinite(v); }

int sched_ok(int s) {
  return s == MPPI_SCHED_AUTO || s == MPPI_SCHED_LANE || s == MPPI_SCHED_WAVE || s == MPPI_SCHED_WIDE ||
         s == MPPI_SCHED_QUAD;
}
// The schedules that spread one sample over several lanes (FP32, h = 32 only).
bool multi_lane(int s) { return s == MPPI_SCHED_WAVE || s == MPPI_SCHED_WIDE; }

// Algorithm 3's zeta = round(K (1 - delta)), half away from zero, in FP64.
int cem_elite_count(int K, float elite) {
  return (int)std::round((double)K * (1.0 - (double)elite));
}

mppi_status validate_config(const mppi_config* c) {
  if (!c) return fail(nullptr, MPPI_E_INVAL, "config is NULL");
  if (c->K < 1 || c->K > kMaxK) return fail(nullptr, MPPI_E_INVAL, "K=%d outside [1, %d]", c->K, kMaxK);
  if (c->T < 1 || c->T > MPPI_T_MAX) return fail(nullptr, MPPI_E_INVAL, "T=%d outside [1, %d]", c->T, MPPI_T_MAX);
  if (!finite(c->dt) || !(c->dt > 0)) return fail(nullptr, MPPI_E_INVAL, "dt must be finite and > 0");
  if (!finite(c->lambda) || !(c->lambda > 0)) return fail(nullptr, MPPI_E_INVAL, "lambda must be finite and > 0");
  if (!finite(c->gamma)) return fail(nullptr, MPPI_E_INVAL, "gamma must be finite");
  for (int i = 0; i < 2; ++i) {
    if (!finite(c->sigma2[i]) || !(c->sigma2[i] > 0))
      return fail(nullptr, MPPI_E_INVAL, "sigma2[%d] must be finite and > 0 (Sigma^-1 must exist)", i);
    if (!finite(c->u_lo[i]) || !finite(c->u_hi[i]) || c->u_lo[i] > c->u_hi[i])
      return fail(nullptr, MPPI_E_INVAL, "clamp bounds u_lo[%d] <= u_hi[%d] must be finite", i, i);
  }
  if (c->sg_window < 1 || c->sg_window % 2 == 0 || c->sg_window > c->T)
    return fail(nullptr, MPPI_E_INVAL, "sg_window=%d must be odd and in [1, T]", c->sg_window);
  if (c->sg_order < 0 || c->sg_order >= c->sg_window)
    return fail(nullptr, MPPI_E_INVAL, "sg_order=%d must be in [0, sg_window)", c->sg_order);
  if (c->precision != MPPI_PREC_FP32 && c->precision != MPPI_PREC_BF16 && c->precision != MPPI_PREC_FP16)
    return fail(nullptr, MPPI_E_INVAL, "unknown precision %d", c->precision);
  if (!sched_ok(c->schedule)) return fail(nullptr, MPPI_E_INVAL, "unknown schedule %d", c->schedule);
  if (!(c->explore >= 0.0f && c->explore <= 1.0f))
    return fail(nullptr, MPPI_E_INVAL, "explore must be in [0, 1]");
  if (c->weighting != MPPI_WEIGHTS_IT && c->weighting != MPPI_WEIGHTS_CEM)
    return fail(nullptr, MPPI_E_INVAL, "unknown weighting %d", c->weighting);
  if (c->weighting == MPPI_WEIGHTS_CEM) {
    if (!(c->elite >= 0.0f && c->elite < 1.0f)) return fail(nullptr, MPPI_E_INVAL, "elite must be in [0, 1)");
    if (cem_elite_count(c->K, c->elite) < 1)
      return fail(nullptr, MPPI_E_INVAL, "round(K (1 - elite)) must be at least 1");
  }
  if (c->k_total == 0) {
    if (c->k_base != 0) return fail(nullptr, MPPI_E_INVAL, "k_base=%u needs k_total (the sharded iteration's size)", c->k_base);
  } else {
    if (c->k_total < 0 || c->k_total > (1 << 30) || (int64_t)c->k_base + c->K > (int64_t)c->k_total)
      return fail(nullptr, MPPI_E_INVAL, "shard k_base=%u, K=%d does not fit k_total=%d (at most 1<<30)", c->k_base,
                  c->K, c->k_total);
    if (c->weighting == MPPI_WEIGHTS_CEM)
      return fail(nullptr, MPPI_E_INVAL, "Algorithm 3 selects over all samples at once; shards merge Algorithm 2 only");
  }
  return MPPI_OK;
}

// Algorithm 1 draws sample k around U while k < (1 - alpha) K: the first
// ceil((1 - alpha) K) samples (evaluated in FP64); the rest are drawn around zero.
int importance_samples(int K, float explore) {
  const double n = std::ceil((1.0 - (double)explore) * (double)K);
  return (int)std::min<double>(std::max<double>(n, 0.0), (double)K);
}

// The same split in a shard's local indices: the iteration's first
// ceil((1 - alpha) k_total) global samples are importance samples.
int importance_samples_shard(const mppi_config& g) {
  if (g.k_total == 0) return importance_samples(g.K, g.explore);
  const double n = std::ceil((1.0 - (double)g.explore) * (double)g.k_total) - (double)g.k_base;
  return (int)std::min<double>(std::max<double>(n, 0.0), (double)g.K);
}

mppi_status validate_cost(const mppi_cost* c) {
  if (!c) return fail(nullptr, MPPI_E_INVAL, "cost is NULL");
  const float v[] = {c->w_map, c->w_speed, c->w_slip, c->v_des, c->crash_cost, c->crash_decay, c->slip_cost};
  for (float x : v)
    if (!finite(x)) return fail(nullptr, MPPI_E_INVAL, "cost weights must be finite");
  if (std::isnan(c->map_thresh) || std::isnan(c->slip_thresh))
    return fail(nullptr, MPPI_E_INVAL, "cost thresholds must not be NaN");
  return MPPI_OK;
}

// Savitzky-Golay rows [T][w]: row t evaluates at t the degree-d least-squares
// polynomial through the w points starting at lo = clamp(t - w/2, 0, T - w).
// Computed by a modified Gram-Schmidt QR of the (scaled) Vandermonde matrix: the
// value at t of the fit is e_0^T R^-1 Q^T y with positions measured from t.
std::vector<float> savgol_rows(int T, int w, int d) {
  std::vector<float> out((size_t)T * w, 0.0f);
  const int n = d + 1;
  const double scale = std::max(1.0, (double)w);
  for (int t = 0; t < T; ++t) {
    const int lo = std::min(std::max(t - w / 2, 0), T - w);
    std::vector<double> Q((size_t)w * n), R((size_t)n * n, 0.0);
    for (int r = 0; r < w; ++r)
      for (int p = 0; p < n; ++p) Q[(size_t)r * n + p] = std::pow((double)(lo + r - t) / scale, p);
    for (int p = 0; p < n; ++p) {
      for (int q = 0; q < p; ++q) {
        double dot = 0;
        for (int r = 0; r < w; ++r) dot += Q[(size_t)r * n + q] * Q[(size_t)r * n + p];
        R[(size_t)q * n + p] = dot;
        for (int r = 0; r < w; ++r) Q[(size_t)r * n + p] -= dot * Q[(size_t)r * n + q];
      }
      double nrm = 0;
      for (int r = 0; r < w; ++r) nrm += Q[(size_t)r * n + p] * Q[(size_t)r * n + p];
      nrm = std::sqrt(nrm);
      R[(size_t)p * n + p] = nrm;
      for (int r = 0; r < w; ++r) Q[(size_t)r * n + p] /= nrm;
    }
    // row 0 of R^-1: solve R^T z = e_0 (forward substitution), then coef = Q z
    std::vector<double> z(n, 0.0);
    for (int p = 0; p < n; ++p) {
      double s = (p == 0) ? 1.0 : 0.0;
      for (int q = 0; q < p; ++q) s -= R[(size_t)q * n + p] * z[q];
      z[p] = s / R[(size_t)p * n + p];
    }
    for (int r = 0; r < w; ++r) {
      double cr = 0;
      for (int p = 0; p < n; ++p) cr += Q[(size_t)r * n + p] * z[p];
      out[(size_t)t * w + r] = (float)cr;
    }
  }
  return out;
}

hipEvent_t take_event(mppi_ctx* c) {
  hipEvent_t e = nullptr;
  if (!c->event_pool.empty()) {
    e = c->event_pool.back();
    c->event_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

mppi_status drain_timing(mppi_ctx* c) {
  for (auto& p : c->pending) {
    HIP_TRY(c, hipEventSynchronize(p.e1));
    float a = 0;
    HIP_TRY(c, hipEventElapsedTime(&a, p.e0, p.e1));
    c->t_ms[p.slot] += a;
    c->t_cnt[p.slot] += 1;
    if (p.slot == 0) c->t_samples.push_back(a);
    c->event_pool.push_back(p.e0);
    c->event_pool.push_back(p.e1);
  }
  c->pending.clear();
  return MPPI_OK;
}

int blocks_for_k(int K, int sched) {
  if (sched == MPPI_SCHED_WAVE) return (K + kWaveSamplesPerBlock - 1) / kWaveSamplesPerBlock;
  if (sched == MPPI_SCHED_WIDE) return (K + kWideSamplesPerBlock - 1) / kWideSamplesPerBlock;
  if (sched == MPPI_SCHED_QUAD) return (K + kQuadSamplesPerBlock - 1) / kQuadSamplesPerBlock;
  return (K + kLaneBlockHost - 1) / kLaneBlockHost;
}

int blocks_for(const mppi_ctx* c, int sched) { return blocks_for_k(c->cfg.K, sched); }

// Compute units of the current device (cached per device).
int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) cus[dev] = n;
  }
  return cus[dev];
}

// The wave schedule.  While the launch fits the device in one block per compute unit
// (the latency-bound regime) and T <= 128, the split kernel runs each block's kinematics
// and cost in a second set of waves one chunk behind the chain; otherwise the wave
// kernel, which keeps each lane's share of the steps (ceil(T/32) of them) in registers
// and is compiled for up to 4 (T <= 128) and up to 8 (T <= 256).
void launch_wave(int G, int T, hipStream_t stream, const RolloutArgs& a) {
  if (T <= kWaveSplitMaxT && G <= device_cus()) {
    const size_t smem = wave_split_smem_bytes(T, a.model);
    if (a.model == kModelBasis)
      hipLaunchKernelGGL((rollout_wave_split_kernel<kModelBasis, false>), dim3(G), dim3(kWaveSplitBlockThreads),
                         smem, stream, a);
    else
      hipLaunchKernelGGL((rollout_wave_split_kernel<kModelNet, false>), dim3(G), dim3(kWaveSplitBlockThreads),
                         smem, stream, a);
    return;
  }
  const size_t smem = wave_smem_bytes(T, a.model);
  if (a.model == kModelBasis) {
    if (T <= 128)
      hipLaunchKernelGGL((rollout_wave_kernel<32, 4, kModelBasis>), dim3(G), dim3(kWaveBlockThreads), smem, stream, a);
    else
      hipLaunchKernelGGL((rollout_wave_kernel<32, 8, kModelBasis>), dim3(G), dim3(kWaveBlockThreads), smem, stream, a);
  } else {
    if (T <= 128)
      hipLaunchKernelGGL((rollout_wave_kernel<32, 4, kModelNet>), dim3(G), dim3(kWaveBlockThreads), smem, stream, a);
    else
      hipLaunchKernelGGL((rollout_wave_kernel<32, 8, kModelNet>), dim3(G), dim3(kWaveBlockThreads), smem, stream, a);
  }
}

// The wide kernel keeps ceil(T/64) steps per lane in registers: up to 2 (T <= 128)
// or up to 4 (T <= 256).
void launch_wide(int G, int T, hipStream_t stream, const RolloutArgs& a) {
  if (T <= 128)
    hipLaunchKernelGGL((rollout_wide_kernel<2>), dim3(G), dim3(kWideBlockThreads), wide_smem_bytes(T), stream, a);
  else
    hipLaunchKernelGGL((rollout_wide_kernel<4>), dim3(G), dim3(kWideBlockThreads), wide_smem_bytes(T), stream, a);
}

// The quad kernel for the network's precision (MPPI_PREC_*, the same codes as the
// kernel's) and width.
void launch_quad(int precision, int hidden, int G, hipStream_t stream, const RolloutArgs& a) {
  const dim3 grid(G), block(kQuadBlockThreads);
#define MPPI_QUAD(P, H) hipLaunchKernelGGL((rollout_quad_kernel<P, H>), grid, block, 0, stream, a)
  if (precision == MPPI_PREC_BF16) {
    if (hidden == 32) MPPI_QUAD(1, 32); else MPPI_QUAD(1, 64);
  } else if (precision == MPPI_PREC_FP16) {
    if (hidden == 32) MPPI_QUAD(2, 32); else MPPI_QUAD(2, 64);
  } else {
    if (hidden == 32) MPPI_QUAD(0, 32); else MPPI_QUAD(0, 64);
  }
#undef MPPI_QUAD
}

// The fields of a rollout launch that follow from the configuration, the cost, the map
// geometry and the dynamics model; the caller sets the buffers and G.
RolloutArgs config_args(const mppi_config& g, const mppi_cost& cost, int H, int W, float ox, float oy,
                        float res, int hidden, int model, const float* x0_host) {
  RolloutArgs a{};
  a.ckpt = nullptr;
  a.ckpt_every = 1;
  a.G = 0;
  a.sg_window = g.sg_window;
  a.update_U = 1;
  for (int i = 0; i < kStateDim; ++i) a.x0[i] = x0_host ? x0_host[i] : 0.0f;
  a.K = g.K;
  a.T = g.T;
  a.K_imp = importance_samples_shard(g);
  a.cem_zeta = g.weighting == MPPI_WEIGHTS_CEM ? cem_elite_count(g.K, g.elite) : 0;
  a.dt = g.dt;
  a.inv_lambda = 1.0f / g.lambda;
  a.gcs0 = g.gamma / g.sigma2[0];
  a.gcs1 = g.gamma / g.sigma2[1];
  a.u_lo0 = g.u_lo[0];
  a.u_lo1 = g.u_lo[1];
  a.u_hi0 = g.u_hi[0];
  a.u_hi1 = g.u_hi[1];
  a.nk.key_lo = (uint32_t)g.seed;
  a.nk.key_hi = (uint32_t)(g.seed >> 32);
  a.nk.iter = 0;
  a.nk.instance = g.instance;
  a.nk.sig0 = std::sqrt(g.sigma2[0]);
  a.nk.sig1 = std::sqrt(g.sigma2[1]);
  a.nk.k_base = g.k_base;
  a.row_out = nullptr;
  a.eps_store = nullptr;
  a.n_steps = 1;
  a.sync = nullptr;
  a.step_base = 0;
  a.hidden = hidden;
  a.model = model;
  a.recede = 0;
  a.u0_out = nullptr;
  a.x_copy = nullptr;
  a.cost.H = H;
  a.cost.W = W;
  a.cost.ox = ox;
  a.cost.oy = oy;
  a.cost.res = res;
  a.cost.w_map = cost.w_map;
  a.cost.w_speed = cost.w_speed;
  a.cost.w_slip = cost.w_slip;
  a.cost.v_des = cost.v_des;
  a.cost.crash_cost = cost.crash_cost;
  a.cost.map_thresh = cost.map_thresh;
  a.cost.slip_cost = cost.slip_cost;
  a.cost.slip_thresh = cost.slip_thresh;
  return a;
}

RolloutArgs rollout_args(const mppi_ctx* c, const float* x0_host, const float* x0_dev) {
  RolloutArgs a = config_args(c->cfg, c->cost, c->H, c->W, c->ox, c->oy, c->res, c->hidden, c->model, x0_host);
  a.U = c->d_U;
  a.map = c->d_map;
  a.params = c->d_params;
  a.decay = c->d_decay;
  a.x0_dev = x0_dev;
  a.part2 = c->d_part2;
  a.cnt = c->d_cnt;
  a.sg = c->d_sg;
  a.Uout = c->d_U;
  a.stats = c->d_stats;
  a.status = c->d_status;
  a.S = c->d_S;
  a.part = c->d_part;
  a.D = c->d_D;
  a.eps_store = c->d_eps;
  a.nk.iter = c->iter;
  a.iter_dev = c->d_iter;
  a.nk.sig0 = c->sig[0];
  a.nk.sig1 = c->sig[1];
  return a;
}

// The schedule the automatic choice resolves to for the network of width h (measured
// on MI355X at T = 100: the 32-lane schedule is fastest while the chains are few and
// latency-bound, the matrix-core quad schedule once K fills the device).
int auto_schedule_net(const mppi_config& g, int h) {
  if (g.schedule != MPPI_SCHED_AUTO) return g.schedule;
  return (g.precision == MPPI_PREC_FP32 && h == 32 && g.K <= kWaveAutoMaxK) ? MPPI_SCHED_WAVE : MPPI_SCHED_QUAD;
}

// Launch the rollout kernel of schedule `sched` (resolved, not AUTO) over G blocks.
// The caller has checked that the schedule serves the model, width and precision.
hipError_t launch_rollout(int sched, int precision, int G, hipStream_t stream, const RolloutArgs& a) {
  if (sched == MPPI_SCHED_WAVE) {
    launch_wave(G, a.T, stream, a);
  } else if (sched == MPPI_SCHED_WIDE) {
    launch_wide(G, a.T, stream, a);
  } else if (sched == MPPI_SCHED_QUAD) {
    launch_quad(precision, a.hidden, G, stream, a);
  } else {
    hipError_t e = launch_lane(precision, a.hidden, dim3(G), stream, a);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// Enqueue one iteration: rollout kernel, then weights/update kernel.
// One launch: an iteration from x0 (host value or device pointer).  With recede set,
// also the shift of U and the plant step of the state in x0_dev (in place), u_0 to
// u0_out and the new state to x_copy (both device, nullable).
mppi_status enqueue_iteration(mppi_ctx* c, const float* x0_host, const float* x0_dev, bool recede = false,
                              float* u0_out = nullptr, float* x_copy = nullptr, float* row_out = nullptr) {
  if (!c->have_map || !c->have_dyn)
    return fail(c, MPPI_E_STATE, "set the cost map and the dynamics before iterating");
  const int sched = c->schedule;
  const int G = blocks_for(c, sched);
  if (G > c->part_cap) return fail(c, MPPI_E_INVAL, "internal: %d partial blocks > capacity %d", G, c->part_cap);
  c->objective_ready = false;
  RolloutArgs a = rollout_args(c, x0_host, x0_dev);
  a.G = G;
  a.recede = recede ? 1 : 0;
  a.u0_out = u0_out;
  a.x_copy = x_copy;
  a.row_out = row_out;
  if (row_out && (a.cem_zeta > 0 || recede))
    return fail(c, MPPI_E_INVAL, "a shard's partial row is Algorithm 2's and ends no receding step");
  PendingTiming pt{};
  if (c->timing) {
    pt.e0 = take_event(c);
    pt.e1 = take_event(c);
    if (!pt.e0 || !pt.e1) return fail(c, MPPI_E_DEVICE, "hipEventCreate failed");
    HIP_TRY(c, hipEventRecord(pt.e0, c->stream));
  }
  if (sched == MPPI_SCHED_WAVE && c->model == kModelNet && c->hidden != 32)
    return fail(c, MPPI_E_INVAL, "wave schedule supports hidden 32 only");
  if (sched == MPPI_SCHED_WIDE && (c->model != kModelNet || c->hidden != 32))
    return fail(c, MPPI_E_INVAL, "wide schedule supports the h = 32 network only");
  if (sched == MPPI_SCHED_QUAD && c->model != kModelNet)
    return fail(c, MPPI_E_INVAL, "quad schedule supports the network only");
  HIP_TRY(c, launch_rollout(sched, c->cfg.precision, G, c->stream, a));
  // Algorithm 3: the rollout launch leaves costs and delta rows; the update follows
  if (a.cem_zeta > 0) {
    // blocks sharing the elite-row sum: one per ~48 elite rows, at most 8, and never more
    // than the partial rows allocated (their counter a.cnt[0] is zero between launches)
    const int nb = std::max(1, std::min({8, (a.cem_zeta + 47) / 48, c->part_cap}));
    const bool h32 = c->model == kModelNet && c->hidden == 32;   // plant step unrolled
    if (c->cfg.T <= 128) {
      if (h32) hipLaunchKernelGGL((cem_update_kernel<2, 32>), dim3(nb), dim3(kCemBlockThreads), 0, c->stream, a);
      else hipLaunchKernelGGL((cem_update_kernel<2, 0>), dim3(nb), dim3(kCemBlockThreads), 0, c->stream, a);
    } else {
      if (h32) hipLaunchKernelGGL((cem_update_kernel<4, 32>), dim3(nb), dim3(kCemBlockThreads), 0, c->stream, a);
      else hipLaunchKernelGGL((cem_update_kernel<4, 0>), dim3(nb), dim3(kCemBlockThreads), 0, c->stream, a);
    }
    HIP_TRY(c, hipGetLastError());
  }
  if (c->timing) {
    HIP_TRY(c, hipEventRecord(pt.e1, c->stream));
    c->pending.push_back(pt);
    if (c->pending.size() >= 512) {
      mppi_status st = drain_timing(c);
      if (st != MPPI_OK) return st;
    }
  }
  c->iter += 1;
  return MPPI_OK;
}

// Whether n receding steps can run as one multi-step launch of the split wave kernel:
// the wave schedule's split form (T <= 128) with its rollout blocks and one merger block
// per merge group fitting one block per compute unit (K <= 1920 on 256 CUs), Algorithm
// 2's weights, and a device that launches cooperatively (every block resident at once).
bool multi_step_ok(const mppi_ctx* c) {
  if (c->schedule != MPPI_SCHED_WAVE || c->cfg.weighting != MPPI_WEIGHTS_IT || c->cfg.T > kWaveSplitMaxT) return false;
  // the rollout blocks and one merger block per merge group, one block per compute unit;
  // a group's arrival words and the group words are each polled by one wave's lanes
  const int G = blocks_for(c, MPPI_SCHED_WAVE);
  if (G + merge_groups(G) > device_cus() || merge_group_size(G) > 64 || merge_groups(G) > 64) return false;
  int coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device) != hipSuccess) return false;
  return coop != 0;
}

// n receding-horizon steps on the state in x_dev (device, updated in place): u_0 of step i
// to u_hist[2i..] and the state after step i to x_hist[7i..] (device, nullable).  One
// cooperative launch when multi_step_ok, else one launch per step; the results are the
// same bit for bit.
mppi_status enqueue_receding_steps(mppi_ctx* c, float* x_dev, int n, float* u_hist, float* x_hist) {
  if (!c->have_map || !c->have_dyn)
    return fail(c, MPPI_E_STATE, "set the cost map and the dynamics before iterating");
  if (n <= 0) return MPPI_OK;
  if (n == 1 || !multi_step_ok(c)) {
    for (int i = 0; i < n; ++i) {
      mppi_status st = enqueue_iteration(c, nullptr, x_dev, true, u_hist ? u_hist + 2 * i : nullptr,
                                         x_hist ? x_hist + kStateDim * i : nullptr);
      if (st != MPPI_OK) return st;
    }
    return MPPI_OK;
  }
  const int G = blocks_for(c, MPPI_SCHED_WAVE);
  if (G > c->part_cap) return fail(c, MPPI_E_INVAL, "internal: %d partial blocks > capacity %d", G, c->part_cap);
  const int ngrp = merge_groups(G);
  if (ngrp > c->ngrp_cap) return fail(c, MPPI_E_INVAL, "internal: %d merge groups > capacity %d", ngrp, c->ngrp_cap);
  c->objective_ready = false;
  RolloutArgs a = rollout_args(c, nullptr, x_dev);
  a.G = G;
  a.recede = 1;
  a.u0_out = u_hist;
  a.x_copy = x_hist;
  a.n_steps = n;
  a.sync = c->d_sync;
  // polls of a step-signal wait (0: the kernel's default), for tests of the give-up path
  if (const char* e = std::getenv("MPPI_STEP_SPIN_LIMIT")) a.spin_limit = (unsigned)std::strtoul(e, nullptr, 10);
  a.step_base = c->step_count;
  PendingTiming pt{};
  if (c->timing) {
    pt.e0 = take_event(c);
    pt.e1 = take_event(c);
    if (!pt.e0 || !pt.e1) return fail(c, MPPI_E_DEVICE, "hipEventCreate failed");
    HIP_TRY(c, hipEventRecord(pt.e0, c->stream));
  }
  void* args[] = {&a};
  const void* fn = c->model == kModelBasis
                       ? reinterpret_cast<const void*>(&rollout_wave_split_kernel<kModelBasis, true>)
                       : reinterpret_cast<const void*>(&rollout_wave_split_kernel<kModelNet, true>);
  HIP_TRY(c, hipLaunchCooperativeKernel(fn, dim3(G + ngrp), dim3(kWaveSplitBlockThreads), args,
                                        (unsigned)wave_split_smem_bytes(c->cfg.T, c->model), c->stream));
  if (c->timing) {
    HIP_TRY(c, hipEventRecord(pt.e1, c->stream));
    c->pending.push_back(pt);
  }
  c->step_count += (unsigned)n;
  c->iter += (uint32_t)n;
  return MPPI_OK;
}

constexpr int kStatusTimeoutHost = 6;   // the split kernel's status when a wait of a multi-step launch gave up

mppi_status read_status(mppi_ctx* c) {
  int st = 0;
  HIP_TRY(c, hipMemcpyAsync(&st, c->d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (st == MPPI_E_NONFINITE) return fail(c, MPPI_E_NONFINITE, "no sample had a finite cost; U unchanged");
  if (st == kStatusTimeoutHost) {
    // the launch left mid-step; the signal words it wrote hold steps below every later
    // launch's, so only the status is cleared for the next launch
    (void)hipMemsetAsync(c->d_status, 0, sizeof(int), c->stream);
    (void)hipStreamSynchronize(c->stream);
    return fail(c, MPPI_E_DEVICE, "a multi-step receding launch gave up waiting for another block");
  }
  return MPPI_OK;
}

template <class F>
mppi_status guarded(mppi_ctx* c, F&& fn) {
  try {
    return fn();
  } catch (const std::bad_alloc&) {
    return fail(c, MPPI_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(c, MPPI_E_DEVICE, "unexpected internal error");
  }
}

mppi_status launch_plant(mppi_ctx* c, const float* x_in_dev, const float* u_dev, float* x_out_dev,
                         float* x_copy_dev) {
  const mppi_config& g = c->cfg;
  if (c->model == kModelBasis)
    hipLaunchKernelGGL(plant_kernel<0>, dim3(1), dim3(64), 0, c->stream, c->d_params, x_in_dev, u_dev,
                       x_out_dev, x_copy_dev, g.dt, g.u_lo[0], g.u_lo[1], g.u_hi[0], g.u_hi[1]);
  else if (c->hidden == 32)
    hipLaunchKernelGGL(plant_kernel<32>, dim3(1), dim3(64), 0, c->stream, c->d_params, x_in_dev, u_dev,
                       x_out_dev, x_copy_dev, g.dt, g.u_lo[0], g.u_lo[1], g.u_hi[0], g.u_hi[1]);
  else
    hipLaunchKernelGGL(plant_kernel<64>, dim3(1), dim3(64), 0, c->stream, c->d_params, x_in_dev, u_dev,
                       x_out_dev, x_copy_dev, g.dt, g.u_lo[0], g.u_lo[1], g.u_hi[0], g.u_hi[1]);
  HIP_TRY(c, hipGetLastError());
  return MPPI_OK;
}

// Copies n parameter floats to the device (reallocating when the count changes) and
// marks the dynamics as set.  Synchronises.
mppi_status upload_params(mppi_ctx* c, const float* params, size_t n) {
  if (c->d_params && c->n_params != n) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipFree(c->d_params));
    c->d_params = nullptr;
  }
  if (!c->d_params) HIP_TRY(c, hipMalloc(&c->d_params, sizeof(float) * n));
  c->n_params = n;
  HIP_TRY(c, hipMemcpyAsync(c->d_params, params, sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->objective_ready = false;
  c->have_dyn = true;
  return MPPI_OK;
}

void free_all(mppi_ctx* c) {
  float** bufs[] = {&c->d_U, &c->d_map, &c->d_params, &c->d_decay, &c->d_S, &c->d_D, &c->d_eps, &c->d_part, &c->d_part2,
                    &c->d_stats, &c->d_sg, &c->d_x, &c->d_u0, &c->d_hist_u, &c->d_hist_x,
                    &c->d_ckpt, &c->d_gpart, &c->d_gout, &c->d_gred};
  for (float** b : bufs) {
    if (*b) (void)hipFree(*b);
    *b = nullptr;
  }
  if (c->d_status) (void)hipFree(c->d_status);
  c->d_status = nullptr;
  if (c->d_cnt) (void)hipFree(c->d_cnt);
  c->d_cnt = nullptr;
  if (c->d_iter) (void)hipFree(c->d_iter);
  c->d_iter = nullptr;
  if (c->d_sync) (void)hipFree(c->d_sync);
  c->d_sync = nullptr;
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.e0);
    (void)hipEventDestroy(p.e1);
  }
  c->pending.clear();
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  c->event_pool.clear();
}

}  // namespace

extern "C" {

const char* mppi_last_error(const mppi_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

mppi_status mppi_create(const mppi_config* cfg, const mppi_cost* cost, int device, void* hip_stream,
                        mppi_ctx** out) {
  g_create_error.clear();
  if (!out) return fail(nullptr, MPPI_E_INVAL, "out is NULL");
  *out = nullptr;
  mppi_status st = validate_config(cfg);
  if (st != MPPI_OK) return st;
  st = validate_cost(cost);
  if (st != MPPI_OK) return st;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(nullptr, MPPI_E_DEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(nullptr, MPPI_E_INVAL, "device %d outside [0, %d)", device, ndev);
  mppi_ctx* c = new (std::nothrow) mppi_ctx();
  if (!c) return fail(nullptr, MPPI_E_NOMEM, "host allocation failed");
  st = guarded(c, [&]() -> mppi_status {
    c->cfg = *cfg;
    c->cost = *cost;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    HIP_TRY(c, hipSetDevice(device));
    const int K = cfg->K, T = cfg->T;
    c->sig[0] = std::sqrt(cfg->sigma2[0]);
    c->sig[1] = std::sqrt(cfg->sigma2[1]);
    c->schedule = cfg->schedule;
    c->part_cap = std::max({blocks_for(c, MPPI_SCHED_LANE), blocks_for(c, MPPI_SCHED_WAVE),
                            blocks_for(c, MPPI_SCHED_WIDE), blocks_for(c, MPPI_SCHED_QUAD)});
    HIP_TRY(c, hipMalloc(&c->d_U, sizeof(float) * 2 * T));
    HIP_TRY(c, hipMemsetAsync(c->d_U, 0, sizeof(float) * 2 * T, c->stream));
    HIP_TRY(c, hipMalloc(&c->d_S, sizeof(float) * K));
    if (cfg->weighting == MPPI_WEIGHTS_CEM) HIP_TRY(c, hipMalloc(&c->d_D, sizeof(float) * (size_t)K * 2 * T));
    HIP_TRY(c, hipMalloc(&c->d_part, sizeof(float) * (size_t)c->part_cap * (2 + 2 * T)));
    const int ngrp_cap = std::max({merge_groups(blocks_for(c, MPPI_SCHED_LANE)),
                                   merge_groups(blocks_for(c, MPPI_SCHED_WAVE)),
                                   merge_groups(blocks_for(c, MPPI_SCHED_WIDE)),
                                   merge_groups(blocks_for(c, MPPI_SCHED_QUAD))});
    // two sets of group rows: a multi-step receding launch alternates them by step
    HIP_TRY(c, hipMalloc(&c->d_part2, sizeof(float) * (size_t)2 * ngrp_cap * (2 + 2 * T)));
    c->ngrp_cap = ngrp_cap;
    HIP_TRY(c, hipMalloc(&c->d_cnt, sizeof(unsigned) * (ngrp_cap + 1)));
    HIP_TRY(c, hipMemsetAsync(c->d_cnt, 0, sizeof(unsigned) * (ngrp_cap + 1), c->stream));
    HIP_TRY(c, hipMalloc(&c->d_stats, sizeof(float) * (2 + 2 * T)));
    HIP_TRY(c, hipMemsetAsync(c->d_stats, 0, sizeof(float) * (2 + 2 * T), c->stream));
    HIP_TRY(c, hipMalloc(&c->d_status, sizeof(int)));
    HIP_TRY(c, hipMemsetAsync(c->d_status, 0, sizeof(int), c->stream));
    HIP_TRY(c, hipMalloc(&c->d_iter, sizeof(unsigned)));
    HIP_TRY(c, hipMemsetAsync(c->d_iter, 0, sizeof(unsigned), c->stream));
    HIP_TRY(c, hipMalloc(&c->d_sync, sizeof(unsigned) * kSyncWords(c->part_cap)));
    HIP_TRY(c, hipMemsetAsync(c->d_sync, 0, sizeof(unsigned) * kSyncWords(c->part_cap), c->stream));
    HIP_TRY(c, hipMalloc(&c->d_x, sizeof(float) * kStateDim));
    HIP_TRY(c, hipMalloc(&c->d_u0, sizeof(float) * 2));
    std::vector<float> decay(T + 1);
    for (int t = 0; t <= T; ++t) decay[t] = (float)std::pow((double)cost->crash_decay, (double)t);
    HIP_TRY(c, hipMalloc(&c->d_decay, sizeof(float) * (T + 1)));
    HIP_TRY(c, hipMemcpy(c->d_decay, decay.data(), sizeof(float) * (T + 1), hipMemcpyHostToDevice));
    if (cfg->sg_window > 1) {
      std::vector<float> rows = savgol_rows(T, cfg->sg_window, cfg->sg_order);
      HIP_TRY(c, hipMalloc(&c->d_sg, sizeof(float) * rows.size()));
      HIP_TRY(c, hipMemcpy(c->d_sg, rows.data(), sizeof(float) * rows.size(), hipMemcpyHostToDevice));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MPPI_OK;
  });
  if (st != MPPI_OK) {
    g_create_error = c->err;
    free_all(c);
    delete c;
    return st;
  }
  *out = c;
  return MPPI_OK;
}

void mppi_destroy(mppi_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_all(ctx);
  delete ctx;
}

mppi_status mppi_set_costmap(mppi_ctx* c, const float* map, int32_t H, int32_t W, float origin_x,
                             float origin_y, float resolution) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!map) return fail(c, MPPI_E_INVAL, "map is NULL");
    if (H < 2 || W < 2 || (int64_t)H * W > (int64_t)1 << 30)
      return fail(c, MPPI_E_INVAL, "map size %d x %d unsupported", H, W);
    if (!finite(origin_x) || !finite(origin_y) || !finite(resolution) || !(resolution > 0))
      return fail(c, MPPI_E_INVAL, "origin must be finite and resolution > 0");
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->d_map && (c->H != H || c->W != W)) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      HIP_TRY(c, hipFree(c->d_map));
      c->d_map = nullptr;
    }
    if (!c->d_map) HIP_TRY(c, hipMalloc(&c->d_map, sizeof(float) * (size_t)H * W));
    HIP_TRY(c, hipMemcpyAsync(c->d_map, map, sizeof(float) * (size_t)H * W, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->objective_ready = false;
    c->H = H;
    c->W = W;
    c->ox = origin_x;
    c->oy = origin_y;
    c->res = resolution;
    c->have_map = true;
    return MPPI_OK;
  });
}

mppi_status mppi_set_basis_dynamics(mppi_ctx* c, const float* theta) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!theta) return fail(c, MPPI_E_INVAL, "theta is NULL");
    if (c->cfg.precision != MPPI_PREC_FP32)
      return fail(c, MPPI_E_INVAL, "the basis-function model runs in FP32 (precision must be FP32)");
    if (c->cfg.schedule == MPPI_SCHED_WIDE || c->cfg.schedule == MPPI_SCHED_QUAD)
      return fail(c, MPPI_E_INVAL, "the basis-function model runs on the lane and wave schedules");
    const size_t n = (size_t)kNumBasisHost * 4;
    for (size_t i = 0; i < n; ++i)
      if (!finite(theta[i])) return fail(c, MPPI_E_INVAL, "Theta entry %zu is not finite", i);
    HIP_TRY(c, hipSetDevice(c->device));
    mppi_status st = upload_params(c, theta, n);
    if (st != MPPI_OK) return st;
    c->model = kModelBasis;
    if (c->cfg.schedule == MPPI_SCHED_AUTO)
      c->schedule = c->cfg.K <= kWaveAutoMaxK ? MPPI_SCHED_WAVE : MPPI_SCHED_LANE;
    return MPPI_OK;
  });
}

mppi_status mppi_set_dynamics(mppi_ctx* c, const int32_t dims[4], const float* params) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!dims || !params) return fail(c, MPPI_E_INVAL, "dims or params is NULL");
    const int h = dims[1];
    if (dims[0] != 6 || dims[3] != 4 || dims[1] != dims[2] || (h != 32 && h != 64))
      return fail(c, MPPI_E_INVAL, "dims must be {6, h, h, 4} with h = 32 or 64");
    if (c->cfg.precision != MPPI_PREC_FP32 && multi_lane(c->cfg.schedule))
      return fail(c, MPPI_E_INVAL, "the wave and wide schedules run the FP32 network only");
    if (multi_lane(c->cfg.schedule) && h != 32)
      return fail(c, MPPI_E_INVAL, "the wave and wide schedules support h = 32 only");
    const size_t n = (size_t)6 * h + h + (size_t)h * h + h + 4 * (size_t)h + 4;
    for (size_t i = 0; i < n; ++i)
      if (!finite(params[i])) return fail(c, MPPI_E_INVAL, "parameter %zu is not finite", i);
    HIP_TRY(c, hipSetDevice(c->device));
    mppi_status st = upload_params(c, params, n);
    if (st != MPPI_OK) return st;
    c->hidden = h;
    c->model = kModelNet;
    c->schedule = auto_schedule_net(c->cfg, h);
    if (c->schedule == MPPI_SCHED_QUAD && !c->d_eps)   // the quad tiles' noise, 8 bytes per sample and step
      HIP_TRY(c, hipMalloc(&c->d_eps, sizeof(float) * 2 * (size_t)blocks_for(c, MPPI_SCHED_QUAD) *
                                          kQuadSamplesPerBlock * c->cfg.T));
    return MPPI_OK;
  });
}

mppi_status mppi_set_controls(mppi_ctx* c, const float* U) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!U) return fail(c, MPPI_E_INVAL, "U is NULL");
    for (int i = 0; i < 2 * c->cfg.T; ++i)
      if (!finite(U[i])) return fail(c, MPPI_E_INVAL, "U[%d] is not finite", i);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(c->d_U, U, sizeof(float) * 2 * c->cfg.T, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->objective_ready = false;
    return MPPI_OK;
  });
}

mppi_status mppi_iterate(mppi_ctx* c, const float x0[7], float* costs_out) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!x0) return fail(c, MPPI_E_INVAL, "x0 is NULL");
    for (int i = 0; i < kStateDim; ++i)
      if (!finite(x0[i])) return fail(c, MPPI_E_INVAL, "x0[%d] is not finite", i);
    HIP_TRY(c, hipSetDevice(c->device));
    mppi_status st = enqueue_iteration(c, x0, nullptr);
    if (st != MPPI_OK) return st;
    if (!costs_out) return MPPI_OK;
    HIP_TRY(c, hipMemcpyAsync(costs_out, c->d_S, sizeof(float) * c->cfg.K, hipMemcpyDeviceToHost, c->stream));
    return read_status(c);
  });
}

mppi_status mppi_iterate_device(mppi_ctx* c, const float* x0_dev) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!x0_dev) return fail(c, MPPI_E_INVAL, "x0_dev is NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    return enqueue_iteration(c, nullptr, x0_dev);
  });
}

mppi_status mppi_get_controls(mppi_ctx* c, float* U_out) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!U_out) return fail(c, MPPI_E_INVAL, "U_out is NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(U_out, c->d_U, sizeof(float) * 2 * c->cfg.T, hipMemcpyDeviceToHost, c->stream));
    return read_status(c);
  });
}

mppi_status mppi_shift(mppi_ctx* c, float u0_out[2]) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!u0_out) return fail(c, MPPI_E_INVAL, "u0_out is NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(shift_kernel, dim3(1), dim3(512), 0, c->stream, c->d_U, c->cfg.T, c->d_u0);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(u0_out, c->d_u0, sizeof(float) * 2, hipMemcpyDeviceToHost, c->stream));
    return read_status(c);
  });
}

mppi_status mppi_plant_step(mppi_ctx* c, const float x[7], const float u[2], float x_out[7]) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!x || !u || !x_out) return fail(c, MPPI_E_INVAL, "NULL argument");
    if (!c->have_dyn) return fail(c, MPPI_E_STATE, "set the dynamics first");
    HIP_TRY(c, hipSetDevice(c->device));
    float buf[9];
    std::memcpy(buf, x, 7 * sizeof(float));
    std::memcpy(buf + 7, u, 2 * sizeof(float));
    // the device state buffer d_x (7) and d_u0 (2) are reused as staging
    HIP_TRY(c, hipMemcpyAsync(c->d_x, buf, 7 * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_u0, buf + 7, 2 * sizeof(float), hipMemcpyHostToDevice, c->stream));
    mppi_status st = launch_plant(c, c->d_x, c->d_u0, c->d_x, nullptr);
    if (st != MPPI_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(x_out, c->d_x, 7 * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MPPI_OK;
  });
}

mppi_status mppi_costmap_values(mppi_ctx* c, const float* xy, int32_t n, float* h_out) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!xy || !h_out || n < 0 || n > (1 << 24)) return fail(c, MPPI_E_INVAL, "bad xy, h_out or n");
    if (!c->have_map) return fail(c, MPPI_E_STATE, "set the cost map first");
    for (int i = 0; i < 2 * n; ++i)
      if (!finite(xy[i])) return fail(c, MPPI_E_INVAL, "position %d is not finite", i / 2);
    if (n == 0) return MPPI_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    float* d = nullptr;
    HIP_TRY(c, hipMalloc(&d, sizeof(float) * 3 * (size_t)n));
    const RolloutArgs a = rollout_args(c, nullptr, nullptr);
    hipError_t e = hipMemcpyAsync(d, xy, sizeof(float) * 2 * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(costmap_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, a.cost, c->d_map, d, n,
                         d + 2 * (size_t)n);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(h_out, d + 2 * (size_t)n, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(c, MPPI_E_DEVICE, "cost map lookup: %s", hipGetErrorString(e));
    return MPPI_OK;
  });
}

mppi_status mppi_run_receding(mppi_ctx* c, const float x0[7], int32_t n_iter, float* u_hist,
                              float* x_hist) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!x0 || n_iter < 0 || n_iter > (1 << 20)) return fail(c, MPPI_E_INVAL, "bad x0 or n_iter");
    for (int i = 0; i < kStateDim; ++i)
      if (!finite(x0[i])) return fail(c, MPPI_E_INVAL, "x0[%d] is not finite", i);
    if (!c->have_map || !c->have_dyn) return fail(c, MPPI_E_STATE, "set the cost map and the dynamics first");
    HIP_TRY(c, hipSetDevice(c->device));
    if (n_iter + 1 > c->hist_cap) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      if (c->d_hist_u) HIP_TRY(c, hipFree(c->d_hist_u));
      if (c->d_hist_x) HIP_TRY(c, hipFree(c->d_hist_x));
      c->d_hist_u = c->d_hist_x = nullptr;
      c->hist_cap = n_iter + 1;
      HIP_TRY(c, hipMalloc(&c->d_hist_u, sizeof(float) * 2 * c->hist_cap));
      HIP_TRY(c, hipMalloc(&c->d_hist_x, sizeof(float) * 7 * c->hist_cap));
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_x, x0, 7 * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_hist_x, x0, 7 * sizeof(float), hipMemcpyHostToDevice, c->stream));
    int nonfinite = 0;
    mppi_status st = enqueue_receding_steps(c, c->d_x, n_iter, c->d_hist_u, c->d_hist_x + 7);
    if (st != MPPI_OK) return st;
    if (u_hist && n_iter > 0)
      HIP_TRY(c, hipMemcpyAsync(u_hist, c->d_hist_u, sizeof(float) * 2 * n_iter, hipMemcpyDeviceToHost, c->stream));
    if (x_hist)
      HIP_TRY(c, hipMemcpyAsync(x_hist, c->d_hist_x, sizeof(float) * 7 * (n_iter + 1), hipMemcpyDeviceToHost, c->stream));
    (void)nonfinite;
    return read_status(c);
  });
}

mppi_status mppi_get_stats(mppi_ctx* c, float* rho, float* eta, float* delta_out) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    HIP_TRY(c, hipSetDevice(c->device));
    std::vector<float> buf(2 + 2 * c->cfg.T);
    HIP_TRY(c, hipMemcpyAsync(buf.data(), c->d_stats, sizeof(float) * buf.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (rho) *rho = buf[0];
    if (eta) *eta = buf[1];
    if (delta_out) std::memcpy(delta_out, buf.data() + 2, sizeof(float) * 2 * c->cfg.T);
    return MPPI_OK;
  });
}

mppi_status mppi_get_noise(mppi_ctx* c, uint32_t iter, float* eps_out) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!eps_out) return fail(c, MPPI_E_INVAL, "eps_out is NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t n = (size_t)c->cfg.K * c->cfg.T;
    float* d = nullptr;
    HIP_TRY(c, hipMalloc(&d, sizeof(float) * 2 * n));
    NoiseKey nk{(uint32_t)c->cfg.seed, (uint32_t)(c->cfg.seed >> 32), iter, c->cfg.instance, c->sig[0], c->sig[1],
                c->cfg.k_base};
    hipLaunchKernelGGL(noise_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, nk, c->cfg.K,
                       c->cfg.T, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(eps_out, d, sizeof(float) * 2 * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(c, MPPI_E_DEVICE, "noise dump: %s", hipGetErrorString(e));
    return MPPI_OK;
  });
}

mppi_status mppi_get_iteration(mppi_ctx* c, uint32_t* iter) {
  if (!c || !iter) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    HIP_TRY(c, hipSetDevice(c->device));
    unsigned v = 0;
    HIP_TRY(c, hipMemcpyAsync(&v, c->d_iter, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->iter = v;
    *iter = v;
    return MPPI_OK;
  });
}

mppi_status mppi_set_iteration(mppi_ctx* c, uint32_t iter) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    HIP_TRY(c, hipSetDevice(c->device));
    unsigned v = iter;
    HIP_TRY(c, hipMemcpyAsync(c->d_iter, &v, sizeof(unsigned), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->iter = iter;
    return MPPI_OK;
  });
}

mppi_status mppi_get_timing_samples(mppi_ctx* c, float* ms_out, int32_t cap, int32_t* n_out) {
  if (!c || !n_out || cap < 0 || (cap > 0 && !ms_out)) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    mppi_status st = drain_timing(c);
    if (st != MPPI_OK) return st;
    const int32_t n = (int32_t)std::min<size_t>((size_t)cap, c->t_samples.size());
    for (int32_t i = 0; i < n; ++i) ms_out[i] = c->t_samples[i];
    *n_out = (int32_t)c->t_samples.size();
    return MPPI_OK;
  });
}

mppi_status mppi_step_device(mppi_ctx* c, float* x_dev, float* u0_out_dev) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!x_dev) return fail(c, MPPI_E_INVAL, "x_dev is NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    return enqueue_iteration(c, nullptr, x_dev, true, u0_out_dev, nullptr);
  });
}

mppi_status mppi_iterate_partial(mppi_ctx* c, const float x0[7], float* row_dev, float* costs_out) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!x0 || !row_dev) return fail(c, MPPI_E_INVAL, "x0 or row_dev is NULL");
    for (int i = 0; i < kStateDim; ++i)
      if (!finite(x0[i])) return fail(c, MPPI_E_INVAL, "x0[%d] is not finite", i);
    if (c->cfg.weighting != MPPI_WEIGHTS_IT)
      return fail(c, MPPI_E_INVAL, "a shard's partial row is Algorithm 2's (MPPI_WEIGHTS_IT)");
    HIP_TRY(c, hipSetDevice(c->device));
    mppi_status st = enqueue_iteration(c, x0, nullptr, false, nullptr, nullptr, row_dev);
    if (st != MPPI_OK || !costs_out) return st;
    HIP_TRY(c, hipMemcpyAsync(costs_out, c->d_S, sizeof(float) * c->cfg.K, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MPPI_OK;
  });
}

mppi_status mppi_merge_update(mppi_ctx* c, const float* rows_dev, int32_t n_rows) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!rows_dev || n_rows < 1 || n_rows > 65536)
      return fail(c, MPPI_E_INVAL, "need rows_dev and 1..65536 rows");
    HIP_TRY(c, hipSetDevice(c->device));
    c->objective_ready = false;
    RolloutArgs a = rollout_args(c, nullptr, nullptr);
    a.iter_dev = nullptr;   // the shards' launches advanced the counter
    a.G = 1;
    hipLaunchKernelGGL(merge_update_kernel, dim3(1), dim3(256), 0, c->stream, a, rows_dev, (int)n_rows);
    HIP_TRY(c, hipGetLastError());
    return MPPI_OK;
  });
}

mppi_status mppi_run_receding_device(mppi_ctx* c, float* x_dev, int32_t n_iter, float* u_hist_dev,
                                     float* x_hist_dev) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!x_dev || n_iter < 0 || n_iter > (1 << 20)) return fail(c, MPPI_E_INVAL, "bad x_dev or n_iter");
    HIP_TRY(c, hipSetDevice(c->device));
    return enqueue_receding_steps(c, x_dev, n_iter, u_hist_dev, x_hist_dev);
  });
}

mppi_status mppi_get_schedule(const mppi_ctx* c, int32_t* schedule) {
  if (!c || !schedule) return MPPI_E_INVAL;
  *schedule = c->schedule;
  return MPPI_OK;
}

mppi_status mppi_set_timing(mppi_ctx* c, int32_t enable) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    mppi_status st = drain_timing(c);
    if (st != MPPI_OK) return st;
    c->timing = enable != 0;
    c->t_ms[0] = c->t_ms[1] = 0;
    c->t_cnt[0] = c->t_cnt[1] = 0;
    c->t_samples.clear();
    return MPPI_OK;
  });
}

mppi_status mppi_get_timing(mppi_ctx* c, double times_ms[2], int64_t counts[2]) {
  if (!c || !times_ms || !counts) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    mppi_status st = drain_timing(c);
    if (st != MPPI_OK) return st;
    times_ms[0] = c->t_ms[0];
    times_ms[1] = c->t_ms[1];
    counts[0] = c->t_cnt[0];
    counts[1] = c->t_cnt[1];
    return MPPI_OK;
  });
}

mppi_status mppi_objective(mppi_ctx* c, const float x0[7], uint32_t iter, int32_t ckpt_every,
                           double* J_out, float* costs_out) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!x0) return fail(c, MPPI_E_INVAL, "x0 is NULL");
    for (int i = 0; i < kStateDim; ++i)
      if (!finite(x0[i])) return fail(c, MPPI_E_INVAL, "x0[%d] is not finite", i);
    if (ckpt_every < 1 || ckpt_every > 16) return fail(c, MPPI_E_INVAL, "ckpt_every=%d outside [1, 16]", ckpt_every);
    if (!c->have_map || !c->have_dyn) return fail(c, MPPI_E_STATE, "set the cost map and the dynamics first");
    if (c->model != kModelNet || c->hidden != 32)
      return fail(c, MPPI_E_INVAL, "the objective gradient supports the h = 32 network only");
    if (c->cfg.explore != 0.0f)
      return fail(c, MPPI_E_INVAL, "the objective is defined for importance samples only (explore = 0)");
    if (c->cfg.weighting != MPPI_WEIGHTS_IT)
      return fail(c, MPPI_E_INVAL, "the objective is defined for Algorithm 2's weights only");
    if (c->cfg.k_total != 0)
      return fail(c, MPPI_E_INVAL, "the objective is evaluated over an unsharded iteration (k_total = 0)");
    HIP_TRY(c, hipSetDevice(c->device));
    const int K = c->cfg.K, T = c->cfg.T;
    const int n_ckpt = T / ckpt_every + 1;
    if (n_ckpt > c->ckpt_cap) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      if (c->d_ckpt) HIP_TRY(c, hipFree(c->d_ckpt));
      c->d_ckpt = nullptr;
      HIP_TRY(c, hipMalloc(&c->d_ckpt, sizeof(float) * (size_t)K * n_ckpt * kCkptStride));
      c->ckpt_cap = n_ckpt;
    }
    const int G = blocks_for(c, MPPI_SCHED_WAVE);
    RolloutArgs a = rollout_args(c, x0, nullptr);
    a.nk.iter = iter;      // an explicit iteration; the counter is neither read nor advanced
    a.iter_dev = nullptr;
    a.ckpt = c->d_ckpt;
    a.ckpt_every = ckpt_every;
    a.G = G;
    a.update_U = 0;
    PendingTiming pt{};
    if (c->timing) {
      pt.e0 = take_event(c);
      pt.e1 = take_event(c);
      if (!pt.e0 || !pt.e1) return fail(c, MPPI_E_DEVICE, "hipEventCreate failed");
      HIP_TRY(c, hipEventRecord(pt.e0, c->stream));
    }
    launch_wave(G, T, c->stream, a);
    HIP_TRY(c, hipGetLastError());
    if (c->timing) {
      HIP_TRY(c, hipEventRecord(pt.e1, c->stream));
      c->pending.push_back(pt);
    }
    float st2[2];
    HIP_TRY(c, hipMemcpyAsync(st2, c->d_stats, sizeof(float) * 2, hipMemcpyDeviceToHost, c->stream));
    if (costs_out) HIP_TRY(c, hipMemcpyAsync(costs_out, c->d_S, sizeof(float) * K, hipMemcpyDeviceToHost, c->stream));
    mppi_status st = read_status(c);
    if (st != MPPI_OK) return st;
    if (J_out) *J_out = (double)st2[0] - (double)c->cfg.lambda * std::log((double)st2[1] / (double)K);
    c->objective_ready = true;
    c->obj_ckpt_every = ckpt_every;
    c->obj_iter = iter;
    return MPPI_OK;
  });
}

mppi_status mppi_objective_backward(mppi_ctx* c, float* dJdU, float* dJdtheta) {
  if (!c) return MPPI_E_INVAL;
  return guarded(c, [&]() -> mppi_status {
    if (!c->objective_ready) return fail(c, MPPI_E_STATE, "evaluate mppi_objective first");
    HIP_TRY(c, hipSetDevice(c->device));
    const int K = c->cfg.K, T = c->cfg.T, C = c->obj_ckpt_every;
    const int G = blocks_for(c, MPPI_SCHED_WAVE);
    const size_t stride = (size_t)kNP32Host + 2 * T;
    if (!c->d_gpart) {
      HIP_TRY(c, hipMalloc(&c->d_gpart, sizeof(float) * (size_t)c->part_cap * stride));
      HIP_TRY(c, hipMalloc(&c->d_gout, sizeof(float) * stride));
      HIP_TRY(c, hipMalloc(&c->d_gred, sizeof(float) * kGradChunks * stride));
    }
    AdjointArgs a{};
    RolloutArgs r = rollout_args(c, nullptr, nullptr);
    a.U = c->d_U;
    a.map = c->d_map;
    a.params = c->d_params;
    a.decay = c->d_decay;
    a.S = c->d_S;
    a.stats = c->d_stats;
    a.ckpt = c->d_ckpt;
    a.gpart = c->d_gpart;
    a.K = K;
    a.T = T;
    a.ckpt_every = C;
    a.n_ckpt = T / C + 1;
    a.dt = c->cfg.dt;
    a.inv_lambda = 1.0f / c->cfg.lambda;
    a.u_lo0 = c->cfg.u_lo[0];
    a.u_lo1 = c->cfg.u_lo[1];
    a.u_hi0 = c->cfg.u_hi[0];
    a.u_hi1 = c->cfg.u_hi[1];
    a.nk = r.nk;
    a.nk.iter = c->obj_iter;
    a.cost = r.cost;
    PendingTiming pt{};
    pt.slot = 1;
    if (c->timing) {
      pt.e0 = take_event(c);
      pt.e1 = take_event(c);
      if (!pt.e0 || !pt.e1) return fail(c, MPPI_E_DEVICE, "hipEventCreate failed");
      HIP_TRY(c, hipEventRecord(pt.e0, c->stream));
    }
    hipLaunchKernelGGL(adjoint_wave_kernel, dim3(G), dim3(kWaveBlockThreads), adjoint_smem_bytes(T, C), c->stream, a);
    HIP_TRY(c, hipGetLastError());
    if (c->timing) {
      HIP_TRY(c, hipEventRecord(pt.e1, c->stream));
      c->pending.push_back(pt);
    }
    const int R = std::min(G, kGradChunks);
    hipLaunchKernelGGL(adjoint_reduce_partial_kernel, dim3((unsigned)((stride + 63) / 64), (unsigned)R), dim3(256), 0,
                       c->stream, c->d_gpart, G, (int)stride, R, c->d_gred);
    HIP_TRY(c, hipGetLastError());
    hipLaunchKernelGGL(adjoint_reduce_final_kernel, dim3((unsigned)((stride + 255) / 256)), dim3(256), 0, c->stream,
                       c->d_gred, R, T, c->d_stats, r.gcs0, r.gcs1, c->d_gout);
    HIP_TRY(c, hipGetLastError());
    std::vector<float> out(stride);
    HIP_TRY(c, hipMemcpyAsync(out.data(), c->d_gout, sizeof(float) * stride, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (dJdtheta) std::memcpy(dJdtheta, out.data(), sizeof(float) * kNP32Host);
    if (dJdU) std::memcpy(dJdU, out.data() + kNP32Host, sizeof(float) * 2 * T);
    return MPPI_OK;
  });
}

}  // extern "C"

// ===========================================================================
// Batched form: many independent MPPI problems in one persistent launch
// ===========================================================================
namespace mppi {
__global__ void rollout_batch_kernel(const RolloutArgs*, const int2*, int, const float*, const float*, const float*,
                                     unsigned*);
__global__ void rollout_batch_quad_kernel(const RolloutArgs*, const int2*, int, const float*, const float*,
                                          const float*, unsigned*);
}

struct mppi_batch {
  mppi_config cfg{};
  mppi_cost cost{};
  int device = 0;
  hipStream_t stream = nullptr;
  int n = 0;
  std::vector<int> K, T, G;              // per instance: samples, horizon, tiles of the chosen schedule
  std::vector<size_t> Uoff, Soff, poff, p2off, coff, soff, sgoff, eoff;
  float* d_U = nullptr;
  float* d_S = nullptr;
  float* d_part = nullptr;
  float* d_part2 = nullptr;
  float* d_eps = nullptr;                // quad tiles' noise, per instance [tiles][4][T][16][2]
  unsigned* d_cnt = nullptr;
  float* d_stats = nullptr;
  int* d_status = nullptr;
  float* d_sg = nullptr;
  float* d_decay = nullptr;
  float* d_x0 = nullptr;
  unsigned* d_iter = nullptr;
  float* d_map = nullptr;
  float* d_params = nullptr;
  RolloutArgs* d_args = nullptr;
  int2* d_items = nullptr;
  unsigned* d_queue = nullptr;           // [2]: next work item, blocks that have found the queue empty
  int n_items = 0;
  int H = 0, W = 0;
  float ox = 0, oy = 0, res = 1;
  bool have_map = false, have_dyn = false, ready = false;
  int grid = 0, order = 0;
  double tuned_us = 0;
  bool quad = true;                      // tiles of the quad schedule (64 samples) or the lane one (256)
  bool may_quad = true, may_lane = true; // the schedules the autotuner may choose from
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool own_stream = false;
  std::string err;
};

namespace {

mppi_status bfail(mppi_batch* b, mppi_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) b->err = buf; else g_create_error = buf;
  return st;
}

#define BHIP_TRY(b, expr)                                                                     \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return bfail((b), e_ == hipErrorOutOfMemory ? MPPI_E_NOMEM : MPPI_E_DEVICE, "%s: %s",  \
                   #expr, hipGetErrorString(e_));                                            \
  } while (0)

void batch_free(mppi_batch* b) {
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  b->stream = nullptr;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  void* bufs[] = {b->d_U, b->d_S, b->d_eps, b->d_part, b->d_part2, b->d_cnt, b->d_stats, b->d_status, b->d_sg,
                  b->d_decay, b->d_x0, b->d_iter, b->d_map, b->d_params, b->d_args, b->d_items, b->d_queue};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
}

// Per-instance launch arguments (device pointers into the batch's shared buffers).
std::vector<RolloutArgs> batch_args(const mppi_batch* b) {
  std::vector<RolloutArgs> v(b->n);
  for (int i = 0; i < b->n; ++i) {
    RolloutArgs a{};
    a.U = b->d_U + b->Uoff[i];
    a.map = b->d_map;
    a.params = b->d_params;
    a.decay = b->d_decay;
    a.x0_dev = b->d_x0 + 7 * (size_t)i;
    a.S = b->d_S + b->Soff[i];
    a.part = b->d_part + b->poff[i];
    a.part2 = b->d_part2 + b->p2off[i];
    a.eps_store = b->d_eps ? b->d_eps + b->eoff[i] : nullptr;
    a.cnt = b->d_cnt + b->coff[i];
    a.sg = b->cfg.sg_window > 1 ? b->d_sg + b->sgoff[i] : nullptr;
    a.Uout = b->d_U + b->Uoff[i];
    a.stats = b->d_stats + b->soff[i];
    a.status = b->d_status + i;
    a.G = b->G[i];
    a.sg_window = b->cfg.sg_window;
    a.update_U = 1;
    a.hidden = 32;
    a.model = kModelNet;
    a.iter_dev = b->d_iter + i;
    a.ckpt = nullptr;
    a.ckpt_every = 1;
    a.K = b->K[i];
    a.T = b->T[i];
    a.K_imp = importance_samples(b->K[i], b->cfg.explore);
    a.cem_zeta = 0;
    a.D = nullptr;
    a.dt = b->cfg.dt;
    a.inv_lambda = 1.0f / b->cfg.lambda;
    a.gcs0 = b->cfg.gamma / b->cfg.sigma2[0];
    a.gcs1 = b->cfg.gamma / b->cfg.sigma2[1];
    a.u_lo0 = b->cfg.u_lo[0];
    a.u_lo1 = b->cfg.u_lo[1];
    a.u_hi0 = b->cfg.u_hi[0];
    a.u_hi1 = b->cfg.u_hi[1];
    a.nk.key_lo = (uint32_t)b->cfg.seed;
    a.nk.key_hi = (uint32_t)(b->cfg.seed >> 32);
    a.nk.iter = 0;  // read from iter_dev by the kernel
    a.nk.instance = b->cfg.instance + (uint32_t)i;
    a.nk.sig0 = std::sqrt(b->cfg.sigma2[0]);
    a.nk.sig1 = std::sqrt(b->cfg.sigma2[1]);
    a.cost.H = b->H;
    a.cost.W = b->W;
    a.cost.ox = b->ox;
    a.cost.oy = b->oy;
    a.cost.res = b->res;
    a.cost.w_map = b->cost.w_map;
    a.cost.w_speed = b->cost.w_speed;
    a.cost.w_slip = b->cost.w_slip;
    a.cost.v_des = b->cost.v_des;
    a.cost.crash_cost = b->cost.crash_cost;
    a.cost.map_thresh = b->cost.map_thresh;
    a.cost.slip_cost = b->cost.slip_cost;
    a.cost.slip_thresh = b->cost.slip_thresh;
    v[i] = a;
  }
  return v;
}

// Tiles of the quad schedule (64 samples, four lanes each) or of the lane schedule (256
// samples, one lane each): the per-instance tile counts and launch arguments.  The
// partial rows and counters were allocated for the quad schedule's tile counts, which
// are never smaller.
mppi_status batch_set_tiles(mppi_batch* b, bool quad) {
  const int tile = quad ? kQuadSamplesPerBlock : kLaneBlockHost;
  b->quad = quad;
  b->n_items = 0;
  for (int i = 0; i < b->n; ++i) {
    b->G[i] = (b->K[i] + tile - 1) / tile;
    b->n_items += b->G[i];
  }
  std::vector<RolloutArgs> args = batch_args(b);
  BHIP_TRY(b, hipMemcpy(b->d_args, args.data(), sizeof(RolloutArgs) * args.size(), hipMemcpyHostToDevice));
  return MPPI_OK;
}

// Work items in the given order: 0 = instance by instance, 1 = longest horizon first
// (then largest K), so that the work queue hands out the long tiles first.
std::vector<int2> batch_items(const mppi_batch* b, int order) {
  std::vector<int> idx(b->n);
  for (int i = 0; i < b->n; ++i) idx[i] = i;
  if (order == 1)
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
      return b->T[x] != b->T[y] ? b->T[x] > b->T[y] : b->K[x] > b->K[y];
    });
  std::vector<int2> items;
  items.reserve(b->n_items);
  if (order == 1) {
    // interleave tiles of equal-length instances so that one instance's tiles spread out
    for (int i : idx)
      for (int t = 0; t < b->G[i]; ++t) items.push_back(make_int2(i, t));
  } else {
    for (int i = 0; i < b->n; ++i)
      for (int t = 0; t < b->G[i]; ++t) items.push_back(make_int2(i, t));
  }
  return items;
}

mppi_status batch_launch(mppi_batch* b, int grid) {
  if (b->quad)
    hipLaunchKernelGGL(rollout_batch_quad_kernel, dim3(grid), dim3(kQuadBlockThreads), 0, b->stream,
                       (const RolloutArgs*)b->d_args, (const int2*)b->d_items, b->n_items,
                       (const float*)b->d_map, (const float*)b->d_params, (const float*)b->d_decay, b->d_queue);
  else
    hipLaunchKernelGGL(rollout_batch_kernel, dim3(grid), dim3(kLaneBlockHost), 0, b->stream,
                       (const RolloutArgs*)b->d_args, (const int2*)b->d_items, b->n_items,
                       (const float*)b->d_map, (const float*)b->d_params, (const float*)b->d_decay, b->d_queue);
  BHIP_TRY(b, hipGetLastError());
  return MPPI_OK;
}

// Times each (schedule, order, grid) candidate on the real problem -- the quad
// schedule's 64-sample tiles or the lane schedule's 256-sample tiles (both when the
// configuration leaves the schedule to the library), the work order, and the number of
// persistent blocks -- keeps the fastest, and restores U and the iteration counters so
// tuning leaves no trace in the results.
mppi_status batch_autotune(mppi_batch* b) {
  int ncu = 0;
  BHIP_TRY(b, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device));
  const size_t nU = b->Uoff.back();
  std::vector<float> U0(nU);
  std::vector<unsigned> it0(b->n);
  BHIP_TRY(b, hipMemcpyAsync(U0.data(), b->d_U, sizeof(float) * nU, hipMemcpyDeviceToHost, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(it0.data(), b->d_iter, sizeof(unsigned) * b->n, hipMemcpyDeviceToHost, b->stream));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  hipEvent_t e0, e1;
  BHIP_TRY(b, hipEventCreate(&e0));
  BHIP_TRY(b, hipEventCreate(&e1));
  double best = 1e30;
  int best_grid = 1, best_order = 0;
  bool best_quad = b->may_quad;
  for (int qs = 0; qs < 2; ++qs) {
   const bool quad = qs == 0;
   if (quad ? !b->may_quad : !b->may_lane) continue;
   mppi_status st0 = batch_set_tiles(b, quad);
   if (st0 != MPPI_OK) return st0;
   const int grids[] = {ncu, 2 * ncu, 4 * ncu, 8 * ncu, b->n_items};
   for (int order = 0; order < 2; ++order) {
    std::vector<int2> items = batch_items(b, order);
    BHIP_TRY(b, hipMemcpy(b->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice));
    for (int gsz : grids) {
      const int grid = std::max(1, std::min(gsz, b->n_items));
      mppi_status st = batch_launch(b, grid);   // warm-up
      if (st != MPPI_OK) return st;
      BHIP_TRY(b, hipEventRecord(e0, b->stream));
      for (int r = 0; r < 2; ++r) {
        st = batch_launch(b, grid);
        if (st != MPPI_OK) return st;
      }
      BHIP_TRY(b, hipEventRecord(e1, b->stream));
      BHIP_TRY(b, hipEventSynchronize(e1));
      float ms = 0;
      BHIP_TRY(b, hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_grid = grid;
        best_order = order;
        best_quad = quad;
      }
    }
   }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  mppi_status st1 = batch_set_tiles(b, best_quad);
  if (st1 != MPPI_OK) return st1;
  std::vector<int2> items = batch_items(b, best_order);
  BHIP_TRY(b, hipMemcpy(b->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(b->d_U, U0.data(), sizeof(float) * nU, hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(b->d_iter, it0.data(), sizeof(unsigned) * b->n, hipMemcpyHostToDevice));
  b->grid = best_grid;
  b->order = best_order;
  b->tuned_us = best * 1e3 / 2.0;
  return MPPI_OK;
}

mppi_status batch_prepare(mppi_batch* b) {
  if (b->ready) return MPPI_OK;
  if (!b->have_map || !b->have_dyn) return bfail(b, MPPI_E_STATE, "set the cost map and the dynamics first");
  mppi_status st = batch_autotune(b);
  if (st != MPPI_OK) return st;
  // capture the chosen launch once; every iteration replays it (a new cost map or
  // network re-captures, since their pointers are kernel arguments)
  if (b->exec) BHIP_TRY(b, hipGraphExecDestroy(b->exec));
  b->exec = nullptr;
  if (b->graph) BHIP_TRY(b, hipGraphDestroy(b->graph));
  b->graph = nullptr;
  BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  mppi_status lst = batch_launch(b, b->grid);
  hipError_t le = lst == MPPI_OK ? hipGetLastError() : hipErrorLaunchFailure;
  hipError_t ce = hipStreamEndCapture(b->stream, &b->graph);
  if (le != hipSuccess) return bfail(b, MPPI_E_DEVICE, "capture launch: %s", hipGetErrorString(le));
  if (ce != hipSuccess) return bfail(b, MPPI_E_DEVICE, "end capture: %s", hipGetErrorString(ce));
  BHIP_TRY(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->ready = true;
  return MPPI_OK;
}

}  // namespace

extern "C" {

const char* mppi_batch_last_error(const mppi_batch* b) { return b ? b->err.c_str() : g_create_error.c_str(); }

mppi_status mppi_batch_create(const mppi_config* cfg, const mppi_cost* cost, int32_t n, const int32_t* K,
                              const int32_t* T, int device, void* hip_stream, mppi_batch** out) {
  g_create_error.clear();
  if (!out) return bfail(nullptr, MPPI_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!cfg || !K || !T || n < 1 || n > 65536) return bfail(nullptr, MPPI_E_INVAL, "need 1..65536 instances with K and T");
  if (cfg->k_base != 0 || cfg->k_total != 0)
    return bfail(nullptr, MPPI_E_INVAL, "the batched form's instances are unsharded (k_base = k_total = 0)");
  int sgmax = 0;
  for (int i = 0; i < n; ++i) {
    mppi_config c = *cfg;
    c.K = K[i];
    c.T = T[i];
    c.schedule = MPPI_SCHED_LANE;
    if (validate_config(&c) != MPPI_OK) {
      g_create_error = "instance " + std::to_string(i) + ": " + g_create_error;
      return MPPI_E_INVAL;
    }
    sgmax = std::max(sgmax, T[i] * cfg->sg_window);
  }
  if (cfg->precision != MPPI_PREC_FP32) return bfail(nullptr, MPPI_E_INVAL, "the batched form runs the FP32 network");
  if (cfg->weighting != MPPI_WEIGHTS_IT)
    return bfail(nullptr, MPPI_E_INVAL, "the batched form uses Algorithm 2's weights");
  if (cfg->schedule != MPPI_SCHED_AUTO && cfg->schedule != MPPI_SCHED_LANE && cfg->schedule != MPPI_SCHED_QUAD)
    return bfail(nullptr, MPPI_E_INVAL, "the batched form runs the lane or quad schedule");
  mppi_status st = validate_cost(cost);
  if (st != MPPI_OK) return st;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return bfail(nullptr, MPPI_E_DEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return bfail(nullptr, MPPI_E_INVAL, "device %d outside [0, %d)", device, ndev);
  mppi_batch* b = new (std::nothrow) mppi_batch();
  if (!b) return bfail(nullptr, MPPI_E_NOMEM, "host allocation failed");
  b->cfg = *cfg;
  b->cost = *cost;
  b->device = device;
  b->stream = (hipStream_t)hip_stream;
  b->n = n;
  b->may_quad = cfg->schedule != MPPI_SCHED_LANE;
  b->may_lane = cfg->schedule != MPPI_SCHED_QUAD;
  b->quad = b->may_quad;
  auto body = [&]() -> mppi_status {
    BHIP_TRY(b, hipSetDevice(device));
    if (!b->stream) {   // graph capture needs a stream other than the null stream
      BHIP_TRY(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
      b->own_stream = true;
    }
    size_t u = 0, s = 0, p = 0, p2 = 0, cn = 0, so = 0, sg = 0, ep = 0;
    int items = 0, Tmax = 0;
    for (int i = 0; i < n; ++i) {
      // partial rows and counters for the quad schedule's tiles (at least the lane's)
      const int g = (K[i] + kQuadSamplesPerBlock - 1) / kQuadSamplesPerBlock;
      const int ng = merge_groups(g);
      b->K.push_back(K[i]);
      b->T.push_back(T[i]);
      b->G.push_back(g);
      b->Uoff.push_back(u);
      b->Soff.push_back(s);
      b->poff.push_back(p);
      b->p2off.push_back(p2);
      b->coff.push_back(cn);
      b->soff.push_back(so);
      b->sgoff.push_back(sg);
      b->eoff.push_back(ep);
      u += 2 * (size_t)T[i];
      ep += 2 * (size_t)g * kQuadSamplesPerBlock * T[i];
      s += K[i];
      p += (size_t)g * (2 + 2 * T[i]);
      p2 += (size_t)ng * (2 + 2 * T[i]);
      cn += ng + 1;
      so += 2 + 2 * (size_t)T[i];
      if (cfg->sg_window > 1) sg += (size_t)T[i] * cfg->sg_window;
      items += g;
      Tmax = std::max(Tmax, T[i]);
    }
    b->Uoff.push_back(u);
    b->n_items = items;
    BHIP_TRY(b, hipMalloc(&b->d_U, sizeof(float) * u));
    BHIP_TRY(b, hipMemset(b->d_U, 0, sizeof(float) * u));
    BHIP_TRY(b, hipMalloc(&b->d_S, sizeof(float) * s));
    BHIP_TRY(b, hipMalloc(&b->d_part, sizeof(float) * p));
    BHIP_TRY(b, hipMalloc(&b->d_part2, sizeof(float) * p2));
    if (b->may_quad) BHIP_TRY(b, hipMalloc(&b->d_eps, sizeof(float) * ep));   // 8 bytes per sample and step
    BHIP_TRY(b, hipMalloc(&b->d_cnt, sizeof(unsigned) * cn));
    BHIP_TRY(b, hipMemset(b->d_cnt, 0, sizeof(unsigned) * cn));
    BHIP_TRY(b, hipMalloc(&b->d_stats, sizeof(float) * so));
    BHIP_TRY(b, hipMemset(b->d_stats, 0, sizeof(float) * so));
    BHIP_TRY(b, hipMalloc(&b->d_status, sizeof(int) * n));
    BHIP_TRY(b, hipMemset(b->d_status, 0, sizeof(int) * n));
    BHIP_TRY(b, hipMalloc(&b->d_x0, sizeof(float) * 7 * n));
    BHIP_TRY(b, hipMemset(b->d_x0, 0, sizeof(float) * 7 * n));
    BHIP_TRY(b, hipMalloc(&b->d_iter, sizeof(unsigned) * n));
    BHIP_TRY(b, hipMemset(b->d_iter, 0, sizeof(unsigned) * n));
    BHIP_TRY(b, hipMalloc(&b->d_args, sizeof(RolloutArgs) * n));
    BHIP_TRY(b, hipMalloc(&b->d_items, sizeof(int2) * items));
    BHIP_TRY(b, hipMalloc(&b->d_queue, sizeof(unsigned) * 2));
    BHIP_TRY(b, hipMemset(b->d_queue, 0, sizeof(unsigned) * 2));
    std::vector<float> decay(Tmax + 1);
    for (int t = 0; t <= Tmax; ++t) decay[t] = (float)std::pow((double)cost->crash_decay, (double)t);
    BHIP_TRY(b, hipMalloc(&b->d_decay, sizeof(float) * (Tmax + 1)));
    BHIP_TRY(b, hipMemcpy(b->d_decay, decay.data(), sizeof(float) * (Tmax + 1), hipMemcpyHostToDevice));
    if (cfg->sg_window > 1) {
      BHIP_TRY(b, hipMalloc(&b->d_sg, sizeof(float) * sg));
      for (int i = 0; i < n; ++i) {
        std::vector<float> rows = savgol_rows(T[i], cfg->sg_window, cfg->sg_order);
        BHIP_TRY(b, hipMemcpy(b->d_sg + b->sgoff[i], rows.data(), sizeof(float) * rows.size(), hipMemcpyHostToDevice));
      }
    }
    return MPPI_OK;
  };
  try {
    st = body();
  } catch (...) {
    st = bfail(b, MPPI_E_NOMEM, "host allocation failed");
  }
  if (st != MPPI_OK) {
    g_create_error = b->err;
    batch_free(b);
    delete b;
    return st;
  }
  *out = b;
  return MPPI_OK;
}

void mppi_batch_destroy(mppi_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  batch_free(b);
  delete b;
}

mppi_status mppi_batch_set_costmap(mppi_batch* b, const float* map, int32_t H, int32_t W, float origin_x,
                                   float origin_y, float resolution) {
  if (!b) return MPPI_E_INVAL;
  if (!map || H < 2 || W < 2 || (int64_t)H * W > (int64_t)1 << 30 || !finite(origin_x) || !finite(origin_y) ||
      !finite(resolution) || !(resolution > 0))
    return bfail(b, MPPI_E_INVAL, "bad cost map");
  BHIP_TRY(b, hipSetDevice(b->device));
  if (b->d_map) BHIP_TRY(b, hipFree(b->d_map));
  BHIP_TRY(b, hipMalloc(&b->d_map, sizeof(float) * (size_t)H * W));
  BHIP_TRY(b, hipMemcpy(b->d_map, map, sizeof(float) * (size_t)H * W, hipMemcpyHostToDevice));
  b->H = H;
  b->W = W;
  b->ox = origin_x;
  b->oy = origin_y;
  b->res = resolution;
  b->have_map = true;
  b->ready = false;
  return MPPI_OK;
}

mppi_status mppi_batch_set_dynamics(mppi_batch* b, const int32_t dims[4], const float* params) {
  if (!b) return MPPI_E_INVAL;
  if (!dims || !params || dims[0] != 6 || dims[1] != 32 || dims[2] != 32 || dims[3] != 4)
    return bfail(b, MPPI_E_INVAL, "the batched form runs the {6, 32, 32, 4} network");
  for (int i = 0; i < kNP32Host; ++i)
    if (!finite(params[i])) return bfail(b, MPPI_E_INVAL, "parameter %d is not finite", i);
  BHIP_TRY(b, hipSetDevice(b->device));
  if (!b->d_params) BHIP_TRY(b, hipMalloc(&b->d_params, sizeof(float) * kNP32Host));
  BHIP_TRY(b, hipMemcpy(b->d_params, params, sizeof(float) * kNP32Host, hipMemcpyHostToDevice));
  b->have_dyn = true;
  b->ready = false;
  return MPPI_OK;
}

mppi_status mppi_batch_set_controls(mppi_batch* b, int32_t i, const float* U) {
  if (!b || !U || i < 0 || i >= b->n) return b ? bfail(b, MPPI_E_INVAL, "bad instance or U") : MPPI_E_INVAL;
  BHIP_TRY(b, hipSetDevice(b->device));
  BHIP_TRY(b, hipMemcpyAsync(b->d_U + b->Uoff[i], U, sizeof(float) * 2 * b->T[i], hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  return MPPI_OK;
}

mppi_status mppi_batch_iterate(mppi_batch* b, const float* x0) {
  if (!b) return MPPI_E_INVAL;
  if (!x0) return bfail(b, MPPI_E_INVAL, "x0 is NULL");
  for (int i = 0; i < 7 * b->n; ++i)
    if (!finite(x0[i])) return bfail(b, MPPI_E_INVAL, "x0[%d] is not finite", i);
  BHIP_TRY(b, hipSetDevice(b->device));
  BHIP_TRY(b, hipMemcpyAsync(b->d_x0, x0, sizeof(float) * 7 * b->n, hipMemcpyHostToDevice, b->stream));
  mppi_status st = batch_prepare(b);
  if (st != MPPI_OK) return st;
  BHIP_TRY(b, hipGraphLaunch(b->exec, b->stream));
  return MPPI_OK;
}

mppi_status mppi_batch_get_controls(mppi_batch* b, int32_t i, float* U_out) {
  if (!b || !U_out || i < 0 || i >= b->n) return b ? bfail(b, MPPI_E_INVAL, "bad instance or U_out") : MPPI_E_INVAL;
  BHIP_TRY(b, hipSetDevice(b->device));
  int st = 0;
  BHIP_TRY(b, hipMemcpyAsync(U_out, b->d_U + b->Uoff[i], sizeof(float) * 2 * b->T[i], hipMemcpyDeviceToHost, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(&st, b->d_status + i, sizeof(int), hipMemcpyDeviceToHost, b->stream));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  return st == MPPI_E_NONFINITE ? bfail(b, MPPI_E_NONFINITE, "instance %d: no finite cost", i) : MPPI_OK;
}

mppi_status mppi_batch_get_costs(mppi_batch* b, int32_t i, float* S_out) {
  if (!b || !S_out || i < 0 || i >= b->n) return b ? bfail(b, MPPI_E_INVAL, "bad instance or S_out") : MPPI_E_INVAL;
  BHIP_TRY(b, hipSetDevice(b->device));
  BHIP_TRY(b, hipMemcpyAsync(S_out, b->d_S + b->Soff[i], sizeof(float) * b->K[i], hipMemcpyDeviceToHost, b->stream));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  return MPPI_OK;
}

mppi_status mppi_batch_get_schedule(mppi_batch* b, int32_t* grid, int32_t* order, double* tuned_us,
                                    int32_t* schedule) {
  if (!b) return MPPI_E_INVAL;
  if (schedule) *schedule = b->quad ? MPPI_SCHED_QUAD : MPPI_SCHED_LANE;
  if (grid) *grid = b->grid;
  if (order) *order = b->order;
  if (tuned_us) *tuned_us = b->tuned_us;
  return b->ready ? MPPI_OK : bfail(b, MPPI_E_STATE, "no iteration has run yet");
}

mppi_status mppi_batch_synchronize(mppi_batch* b) {
  if (!b) return MPPI_E_INVAL;
  BHIP_TRY(b, hipSetDevice(b->device));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  return MPPI_OK;
}

}  // extern "C"

// ===========================================================================
// Allocation-free iteration: the launch's scratch in a static device array
// ===========================================================================
namespace {

constexpr int kNaMaxK = 16384;       // samples per call
constexpr int kNaMaxWindow = 31;     // Savitzky-Golay window
constexpr int kNaMaxDevices = 64;
constexpr size_t kNaRow = 2 + 2 * (size_t)MPPI_T_MAX;   // floats per partial row at the largest T
// partial rows of the schedules with the most blocks (8 samples per block)
constexpr int kNaMaxBlocks = (kNaMaxK + kWaveSamplesPerBlock - 1) / kWaveSamplesPerBlock;
constexpr int kNaMaxGroups = merge_groups(kNaMaxBlocks);
constexpr size_t na_round(size_t n) { return (n + 63) / 64 * 64; }   // whole 256-byte lines
// offsets (in 4-byte words) of the regions of the scratch
constexpr size_t kNaPart = 0;                                                    // [G][2 + 2T]
constexpr size_t kNaPart2 = kNaPart + na_round((size_t)kNaMaxBlocks * kNaRow);    // [groups][2 + 2T]
constexpr size_t kNaCnt = kNaPart2 + na_round((size_t)kNaMaxGroups * kNaRow);     // [groups + 1] unsigned
constexpr size_t kNaStats = kNaCnt + na_round((size_t)kNaMaxGroups + 1);          // [2 + 2T]
constexpr size_t kNaStatus = kNaStats + na_round(kNaRow);                         // [1] int
constexpr size_t kNaDecay = kNaStatus + na_round(1);                              // [T + 1]
constexpr size_t kNaSg = kNaDecay + na_round((size_t)MPPI_T_MAX + 1);             // [T][window]
constexpr size_t kNaS = kNaSg + na_round((size_t)MPPI_T_MAX * kNaMaxWindow);      // [K] when S_dev is NULL
constexpr size_t kNaWords = kNaS + na_round((size_t)kNaMaxK);
static_assert(sizeof(float) == sizeof(unsigned) && sizeof(float) == sizeof(int), "word-sized regions");

// The scratch of mppi_iterate_noalloc (kNaWords 4-byte words, about 4.3 MiB), one copy on
// every device the library runs on, held until the process ends.  In host code this name
// is a host-side stand-in, not a device address: host code uses only the address that
// hipGetSymbolAddress returned for the device (NaDevice::ptr).
static __device__ __align__(256) float scratch[kNaWords];

__global__ void na_clear_kernel(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Per device: the scratch's address and which tables it holds.
struct NaDevice {
  bool ready = false;
  float* ptr = nullptr;        // device address of `scratch` on this device
  bool tables = false;         // decay and smoothing tables loaded for the key below
  int T = 0, window = 0, order = 0;
  uint32_t decay_bits = 0;
};
std::mutex g_na_mutex;
NaDevice g_na[kNaMaxDevices];

// Set-up on the current device, once: the scratch's address, and its arrival counters
// zeroed by a kernel (every launch leaves them at zero again).
mppi_status na_setup(NaDevice& d) {
  if (d.ready) return MPPI_OK;
  float* p = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(nullptr, MPPI_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  const int n = kNaMaxGroups + 1;
  hipLaunchKernelGGL(na_clear_kernel, dim3((n + 255) / 256), dim3(256), 0, nullptr,
                     reinterpret_cast<unsigned*>(p + kNaCnt), n);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail(nullptr, MPPI_E_DEVICE, "clearing the scratch counters: %s", hipGetErrorString(e));
  d.ptr = p;
  d.ready = true;
  return MPPI_OK;
}

// The crash-decay and Savitzky-Golay tables of (T, window, order, decay) in the scratch,
// made on the host exactly as mppi_create makes them.  Loaded only when the key changes,
// after a device-wide synchronisation (an earlier call may still be reading them).
mppi_status na_tables(NaDevice& d, const mppi_config& g, const mppi_cost& cost) {
  uint32_t bits = 0;
  std::memcpy(&bits, &cost.crash_decay, sizeof bits);
  const int order = g.sg_window > 1 ? g.sg_order : 0;
  if (d.tables && d.T == g.T && d.window == g.sg_window && d.order == order && d.decay_bits == bits)
    return MPPI_OK;
  d.tables = false;
  float decay[MPPI_T_MAX + 1];
  for (int t = 0; t <= g.T; ++t) decay[t] = (float)std::pow((double)cost.crash_decay, (double)t);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(d.ptr + kNaDecay, decay, sizeof(float) * (g.T + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && g.sg_window > 1) {
    const std::vector<float> rows = savgol_rows(g.T, g.sg_window, g.sg_order);
    e = hipMemcpy(d.ptr + kNaSg, rows.data(), sizeof(float) * rows.size(), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return fail(nullptr, MPPI_E_DEVICE, "loading the scratch tables: %s", hipGetErrorString(e));
  d.tables = true;
  d.T = g.T;
  d.window = g.sg_window;
  d.order = order;
  d.decay_bits = bits;
  return MPPI_OK;
}

mppi_status iterate_noalloc(const mppi_config* cfg, const mppi_cost* cost, int device, void* hip_stream,
                            const float* map_dev, int32_t H, int32_t W, float origin_x, float origin_y,
                            float resolution, const int32_t dims[4], const float* params_dev,
                            const float* x0_dev, uint32_t iter, float* U_dev, float* S_dev, int32_t* status_dev) {
  mppi_status st = validate_config(cfg);
  if (st != MPPI_OK) return st;
  st = validate_cost(cost);
  if (st != MPPI_OK) return st;
  if (cfg->K > kNaMaxK) return fail(nullptr, MPPI_E_INVAL, "K=%d above this entry point's maximum %d", cfg->K, kNaMaxK);
  if (cfg->sg_window > kNaMaxWindow)
    return fail(nullptr, MPPI_E_INVAL, "sg_window=%d above this entry point's maximum %d", cfg->sg_window,
                kNaMaxWindow);
  if (cfg->weighting != MPPI_WEIGHTS_IT)
    return fail(nullptr, MPPI_E_INVAL, "this entry point forms Algorithm 2's weights only");
  if (!map_dev || !dims || !params_dev || !x0_dev || !U_dev)
    return fail(nullptr, MPPI_E_INVAL, "map_dev, dims, params_dev, x0_dev and U_dev must not be NULL");
  if (H < 2 || W < 2 || (int64_t)H * W > (int64_t)1 << 30)
    return fail(nullptr, MPPI_E_INVAL, "map size %d x %d unsupported", H, W);
  if (!finite(origin_x) || !finite(origin_y) || !finite(resolution) || !(resolution > 0))
    return fail(nullptr, MPPI_E_INVAL, "origin must be finite and resolution > 0");
  const int h = dims[1];
  if (dims[0] != 6 || dims[3] != 4 || dims[1] != dims[2] || (h != 32 && h != 64))
    return fail(nullptr, MPPI_E_INVAL, "dims must be {6, h, h, 4} with h = 32 or 64");
  const int sched = auto_schedule_net(*cfg, h);
  if (multi_lane(sched) && (cfg->precision != MPPI_PREC_FP32 || h != 32))
    return fail(nullptr, MPPI_E_INVAL, "the wave and wide schedules run the FP32 h = 32 network only");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(nullptr, MPPI_E_DEVICE, "no HIP device available");
  if (device < 0 || device >= ndev || device >= kNaMaxDevices)
    return fail(nullptr, MPPI_E_INVAL, "device %d outside [0, %d)", device, std::min(ndev, kNaMaxDevices));
  std::lock_guard<std::mutex> lock(g_na_mutex);
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, MPPI_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  NaDevice& d = g_na[device];
  st = na_setup(d);
  if (st != MPPI_OK) return st;
  st = na_tables(d, *cfg, *cost);
  if (st != MPPI_OK) return st;
  RolloutArgs a = config_args(*cfg, *cost, H, W, origin_x, origin_y, resolution, h, kModelNet, nullptr);
  float* p = d.ptr;
  a.U = U_dev;
  a.Uout = U_dev;
  a.map = map_dev;
  a.params = params_dev;
  a.decay = p + kNaDecay;
  a.x0_dev = x0_dev;
  a.S = S_dev ? S_dev : p + kNaS;
  a.part = p + kNaPart;
  a.part2 = p + kNaPart2;
  a.cnt = reinterpret_cast<unsigned*>(p + kNaCnt);
  a.sg = cfg->sg_window > 1 ? p + kNaSg : nullptr;
  a.stats = p + kNaStats;
  a.status = status_dev ? reinterpret_cast<int*>(status_dev) : reinterpret_cast<int*>(p + kNaStatus);
  a.D = nullptr;
  a.nk.iter = iter;
  a.iter_dev = nullptr;
  a.G = blocks_for_k(cfg->K, sched);
  e = launch_rollout(sched, cfg->precision, a.G, (hipStream_t)hip_stream, a);
  if (e != hipSuccess) return fail(nullptr, MPPI_E_DEVICE, "rollout launch: %s", hipGetErrorString(e));
  return MPPI_OK;
}

}  // namespace

extern "C" mppi_status mppi_iterate_noalloc(const mppi_config* cfg, const mppi_cost* cost, int device,
                                            void* hip_stream, const float* map_dev, int32_t H, int32_t W,
                                            float origin_x, float origin_y, float resolution,
                                            const int32_t dims[4], const float* params_dev, const float* x0_dev,
                                            uint32_t iter, float* U_dev, float* S_dev, int32_t* status_dev) {
  g_create_error.clear();
  try {
    return iterate_noalloc(cfg, cost, device, hip_stream, map_dev, H, W, origin_x, origin_y, resolution, dims,
                           params_dev, x0_dev, iter, U_dev, S_dev, status_dev);
  } catch (...) {
    return fail(nullptr, MPPI_E_DEVICE, "unexpected internal error");
  }
}
