/*
 * mppi.h - C ABI of the MI355X (gfx950) MPPI library (libmppi.so).
 *
 * One call of mppi_iterate() is one iteration of the sampling-based MPC of
 * Williams et al., "Information Theoretic Model Predictive Control: Theory and
 * Applications to Autonomous Driving" (arXiv 1707.02342), Algorithm 1 without
 * its last block: draw K perturbation sequences E^k = (eps_0..eps_{T-1}),
 * eps ~ N(0, Sigma); roll every sample through x <- F(x, g(u_t + eps_t));
 * accumulate S_k += c(x) + gamma * u_t^T Sigma^-1 eps_t; form the weights of
 * Algorithm 2; and update U <- U + SGF * sum_k w_k E^k.  mppi_shift() is the
 * last block (send u_0, slide the sequence, u_{T-1} <- (0,0), Table 2).
 *
 * The problem follows the paper's statement: discrete dynamics x_{t+1} = F(x_t, v_t)
 * with v_t ~ N(u_t, Sigma) (Section II, Eq. Dynamics), the state cost
 * S(V; x0) = C(H(V; x0)) (Eq. State-Cost), the importance-sampling control law
 * (Eq. IT-Controls) with the cost shift of Section III-D-1, the decoupled
 * control-cost weight gamma of Section III-D-2, the clamp g of Section III-D-3
 * and Savitzky-Golay smoothing of Section III-D-4.  The vehicle model is the
 * paper's (Section VI-B): state (p_x, p_y, theta, roll, v_x, v_y, theta_dot),
 * control (steer, throttle), kinematic states by explicit Euler and the dynamic
 * states by a 6 -> h -> h -> 4 tanh network (h = 32 is the paper's 1412-parameter
 * network); the cost is the paper's track + speed + stabilising cost
 * (Section VI-C) on a cost map given as a grid.
 *
 * Conventions for every entry point:
 *   - All inputs are COPIED into library-owned device memory; the library never
 *     keeps a caller pointer.  Pointers named *_dev are device pointers valid on
 *     the context's device; all others are host pointers.
 *   - Work is enqueued on the stream given to mppi_create (NULL = the device's
 *     null stream).  Calls that return data to the host synchronise that stream.
 *   - No C++ exception crosses this interface.  Every call returns an
 *     mppi_status; on failure the context's last-error string says why.
 *   - A context belongs to one host thread at a time.
 */
#ifndef MPPI_H
#define MPPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mppi_ctx mppi_ctx;

typedef enum {
  MPPI_OK = 0,
  MPPI_E_INVAL = 1,     /* an argument is out of range or inconsistent            */
  MPPI_E_STATE = 2,     /* call order: cost map / dynamics not set yet            */
  MPPI_E_NOMEM = 3,     /* device allocation failed                               */
  MPPI_E_DEVICE = 4,    /* a HIP runtime call or kernel launch failed             */
  MPPI_E_NONFINITE = 5  /* every sampled cost was non-finite; U was left unchanged */
} mppi_status;

enum { MPPI_PREC_FP32 = 0, MPPI_PREC_BF16 = 1, MPPI_PREC_FP16 = 2 };

/* Trajectory weights: Algorithm 2 (information theoretic, softmin at temperature
 * lambda) or Algorithm 3 (cross entropy: the zeta = round(K (1 - elite)) samples of
 * lowest cost weigh 1/zeta each, ties to the lower sample index, non-finite costs never
 * elite; with fewer than zeta finite costs every finite sample weighs 1/their number). */
enum { MPPI_WEIGHTS_IT = 0, MPPI_WEIGHTS_CEM = 1 };

/* Kernel schedule for the rollout (0 = pick automatically).  LANE: one sample per
 * lane (any K; FP32, BF16 or FP16 network, h = 32 or 64; BF16/FP16 on the matrix
 * cores, 64 samples per instruction group).  WAVE: 32 lanes per sample, two samples per wavefront.  WIDE: 64 lanes (a
 * whole wavefront) per sample.  WAVE and WIDE run the FP32 network with h = 32 and
 * suit a few thousand samples, where one lane per sample leaves most of the device
 * idle.  QUAD: 4 lanes per sample, 16 samples per wavefront, the network on the
 * matrix cores in any precision (h = 32 or 64), for tens of thousands of samples.
 * AUTO: WAVE for the FP32 h = 32 network up to K = 12288, QUAD otherwise. */
enum { MPPI_SCHED_AUTO = 0, MPPI_SCHED_LANE = 1, MPPI_SCHED_WAVE = 2, MPPI_SCHED_WIDE = 3, MPPI_SCHED_QUAD = 4 };

#define MPPI_T_MAX 256
#define MPPI_STATE_DIM 7
#define MPPI_CTRL_DIM 2

/* Algorithm 1 "Given" block: K, T, Sigma, gamma, lambda, g and the SGF.
 * Invalid (MPPI_E_INVAL): K < 1 or K > 1<<22; T < 1 or T > MPPI_T_MAX; dt, lambda
 * not finite and > 0; sigma2[i] not finite and > 0 (Sigma^-1 must exist); gamma not
 * finite; u_lo[i] > u_hi[i]; sg_window even, < 1 or > T; sg_order < 0 or
 * >= sg_window; precision not one of MPPI_PREC_*; schedule not one of MPPI_SCHED_*;
 * explore not in [0, 1]; weighting not one of MPPI_WEIGHTS_*; with MPPI_WEIGHTS_CEM,
 * elite not in [0, 1) or round(K (1 - elite)) < 1 (computed in FP64 from the FP32 value).
 * K-shard form (the sample-level parallelism of Section III-D-5 spread over several
 * devices or contexts): with k_total > 0 the context draws the samples of global indices
 * k_base .. k_base + K - 1 of an iteration of k_total samples.  INVAL: k_total != 0 and
 * k_total < k_base + K (or > 1<<30), k_total == 0 with k_base != 0, or a sharded
 * context with MPPI_WEIGHTS_CEM (Algorithm 3 needs one selection over all samples).
 * Exploration samples (Algorithm 1's alpha and the disturbance discussion of
 * Section IV): sample k (global index) is drawn around zero when
 * k >= ceil((1 - explore) k_total), k_total = K when unsharded.  For every
 * sample delta_t = v_t - u_t enters the running cost as gamma u_t^T Sigma^-1 delta_t
 * (the paper's gamma u^T Sigma^-1 v up to a constant shared by all samples) and the
 * update as U <- U + SGF * sum_k w_k delta_k (Eq. IT-Controls).  With explore = 0,
 * delta = eps. */
typedef struct {
  int32_t K;            /* samples per iteration                                   */
  int32_t T;            /* horizon (time steps)                                    */
  float dt;             /* Euler step of the model, seconds                        */
  float lambda;         /* inverse temperature (Algorithm 2)                       */
  float gamma;          /* control-cost weight, gamma = lambda (1 - alpha)         */
  float sigma2[2];      /* Sigma = diag(sigma2): variances of steer, throttle noise */
  float u_lo[2];        /* clamp g: lower bounds                                   */
  float u_hi[2];        /* clamp g: upper bounds                                   */
  int32_t sg_window;    /* Savitzky-Golay window (odd); 1 = smoothing off          */
  int32_t sg_order;     /* Savitzky-Golay polynomial degree; 0 with window 1       */
  int32_t precision;    /* MPPI_PREC_*: arithmetic of the dynamics network         */
  int32_t schedule;     /* MPPI_SCHED_*                                            */
  uint64_t seed;        /* Philox4x32-10 key (lo, hi 32-bit words)                 */
  uint32_t instance;    /* fourth Philox counter word                              */
  float explore;        /* alpha of Algorithm 1: samples k >= ceil((1 - alpha) K)
                           are drawn around zero (v = eps) instead of around U;
                           0 = every sample around U                              */
  int32_t weighting;    /* MPPI_WEIGHTS_*                                          */
  float elite;          /* Algorithm 3's eliteness threshold (0.8: the best 20 %)  */
  uint32_t k_base;      /* K-shard form: global index of this context's sample 0; the
                           Philox counter's second word is the global index k_base + k */
  int32_t k_total;      /* K-shard form: samples of the whole iteration over all shards
                           (0 = unsharded: this context's K, with k_base = 0)         */
} mppi_config;

/* State cost c(x, t) at the post-step state x_t, t = 1..T (Section VI-C):
 *   w_map * h(p_x, p_y) + crash_cost * fl32(crash_decay^t) * [h > map_thresh]
 *   + w_speed * (v_x - v_des)^2 + w_slip * zeta^2 + slip_cost * [|zeta| > slip_thresh],
 *   zeta = -atan2(v_y, |v_x|)  (side-slip angle).
 * All fields finite except the thresholds, which may be +inf (term off). */
typedef struct {
  float w_map, w_speed, w_slip, v_des;
  float crash_cost, crash_decay, map_thresh;
  float slip_cost, slip_thresh;
} mppi_cost;

/* Create a context on HIP device `device`, enqueueing on `hip_stream` (a
 * hipStream_t, or NULL).  Allocates all device buffers for K and T.  U starts at 0. */
mppi_status mppi_create(const mppi_config* cfg, const mppi_cost* cost, int device,
                        void* hip_stream, mppi_ctx** out);

/* Free everything the context owns.  NULL-safe.  Synchronises its stream. */
void mppi_destroy(mppi_ctx* ctx);

/* Human-readable reason of the last failing call on ctx ("" if none).  With
 * ctx == NULL: the reason of the last mppi_create failure on this thread. */
const char* mppi_last_error(const mppi_ctx* ctx);

/* Cost map h: a [H][W] row-major float grid, cell (i, j) at world
 * (origin_x + j*resolution, origin_y + i*resolution); bilinear interpolation with
 * indices clamped to the map edge (the paper keeps it in texture memory,
 * Section VI-C).  Copied.  INVAL: H or W < 2, resolution not > 0, non-finite origin. */
mppi_status mppi_set_costmap(mppi_ctx* ctx, const float* map, int32_t H, int32_t W,
                             float origin_x, float origin_y, float resolution);

/* Dynamics network f(x_d, g(v)) (Section VI-B-2).  dims = {6, h, h, 4} with
 * h = 32 or 64.  params = W1[h][6], b1[h], W2[h][h], b2[h], W3[4][h], b3[4]
 * (row-major [out][in]); inputs (roll, v_x, v_y, theta_dot, steer, throttle),
 * outputs d/dt of (roll, v_x, v_y, theta_dot).  Copied.  When the schedule resolves to
 * QUAD this allocates, once per context, 8 bytes per sample and step (ceil(K/64) 64 T
 * pairs of floats): the rollouts keep their noise there for the weighted perturbation
 * sum instead of drawing it twice.  INVAL: other dims, non-finite parameters, or a
 * precision the given h does not support.  NOMEM: that buffer could not be allocated. */
mppi_status mppi_set_dynamics(mppi_ctx* ctx, const int32_t dims[4], const float* params);

/* Basis-function dynamics model (Section VI-B-1 and the appendix), in place of the
 * network: f(x_d, g(v)) = Theta^T phi(x_d, g(v)) with the appendix's 25 basis functions
 * (its r is the heading rate theta_dot, its theta the roll).  theta = Theta[25][4]
 * row-major: row i for basis function i + 1, column o for d/dt of (roll, v_x, v_y,
 * theta_dot).  Copied.  Runs in FP32 on the LANE and WAVE schedules (AUTO: WAVE up to
 * K = 12288, LANE above); the last set_*dynamics call chooses the model.
 * INVAL: non-finite entries, precision other than FP32, schedule WIDE or QUAD.  The
 * differentiation form (mppi_objective) and the batched form use the network only. */
mppi_status mppi_set_basis_dynamics(mppi_ctx* ctx, const float* theta);

/* The cost map h at n world positions xy ([n][2] (p_x, p_y), host) into h_out ([n],
 * host), with the rollout kernels' bilinear interpolation (for closed-loop evaluation:
 * where an executed trajectory left the track).  Synchronises.  INVAL: NULL pointers,
 * n outside [0, 1<<24] or a non-finite position.  STATE: no cost map set. */
mppi_status mppi_costmap_values(mppi_ctx* ctx, const float* xy, int32_t n, float* h_out);

/* Replace the nominal control sequence U ([T][2], steer/throttle per step).  Copied. */
mppi_status mppi_set_controls(mppi_ctx* ctx, const float* U);

/* One MPPI iteration from state x0[7] (host).  Enqueued; returns without waiting
 * unless costs_out ([K] host floats, the S_k of this iteration, +inf for a
 * non-finite sample) is given, in which case it synchronises and also reports
 * MPPI_E_NONFINITE.  The Philox counter's third word is the iteration count,
 * which starts at 0 and increments on every call.
 * STATE: map or dynamics not set. */
mppi_status mppi_iterate(mppi_ctx* ctx, const float x0[7], float* costs_out);

/* As mppi_iterate, with x0 read from device memory (7 floats) when the kernel runs. */
mppi_status mppi_iterate_device(mppi_ctx* ctx, const float* x0_dev);

/* Copy U ([T][2]) to the host.  Synchronises.  Returns MPPI_E_NONFINITE if the
 * most recent iteration found no finite cost (U was then left unchanged). */
mppi_status mppi_get_controls(mppi_ctx* ctx, float* U_out);

/* Algorithm 1's last block: u0_out = u_0; u_{t-1} <- u_t; u_{T-1} <- (0, 0).
 * Synchronises.  Returns MPPI_E_NONFINITE like mppi_get_controls. */
mppi_status mppi_shift(mppi_ctx* ctx, float u0_out[2]);

/* Noise-free plant step x_out = F(x, g(u)) with the context's model (FP32, on the
 * GPU).  Synchronises.  Used to drive a receding-horizon loop on a synthetic plant. */
mppi_status mppi_plant_step(mppi_ctx* ctx, const float x[7], const float u[2], float x_out[7]);

/* n_iter receding-horizon steps entirely on the device: iterate from x, shift,
 * then x <- F(x, g(u_0)) (Algorithm 1 on a synthetic plant), launched as
 * mppi_run_receding_device launches them (one multi-step launch where the split wave
 * form applies, else one launch per step).  u_hist ([n_iter][2]) and x_hist ([n_iter+1][7], x_hist[0] = x0) may be NULL.
 * The results equal the host-driven loop mppi_iterate / mppi_shift / mppi_plant_step
 * bit for bit.  Synchronises at the end only. */
mppi_status mppi_run_receding(mppi_ctx* ctx, const float x0[7], int32_t n_iter,
                              float* u_hist, float* x_hist);

/* One receding-horizon control step on device data: iterate from the state in x_dev
 * (device pointer, [7] floats), shift U (u_0 to u0_out_dev, a device pointer to [2]
 * floats, or NULL) and advance x_dev in place by the noise-free plant step.  Enqueues
 * one launch on the context's stream and returns: no synchronisation, no allocation
 * and no host copy, so with timing off it can be captured in a HIP graph and
 * replayed; each replay advances the device-side iteration counter.  x_dev must stay
 * valid until the launch has run.  The iteration's status is read by the next
 * synchronising call (mppi_get_controls, mppi_shift). */
mppi_status mppi_step_device(mppi_ctx* ctx, float* x_dev, float* u0_out_dev);

/* n_iter receding-horizon control steps on device data (Algorithm 1 with its last block
 * on a synthetic plant): each step iterates from the state in x_dev (device, [7],
 * updated in place by the noise-free plant step), shifts U, writes u_0 to u_hist_dev[2i..]
 * and the new state to x_hist_dev[7i..] (device, [n_iter][2] and [n_iter][7], either may
 * be NULL).  Enqueued, no synchronisation, no allocation.  With the wave schedule's split
 * form (T <= 128; its blocks of 8 samples plus one merging block per group of about
 * sqrt(K/8) of them fit one block per compute unit: K <= 1920 on 256 CUs) and Algorithm
 * 2's weights, all n_iter steps run in ONE cooperative launch whose blocks keep the
 * network in registers and run every step's update themselves; otherwise one launch per
 * step.  Either way the results equal n_iter calls of mppi_step_device bit for bit.  The
 * status of the last step (or MPPI_E_DEVICE if a block of the multi-step launch gave up
 * waiting for another: U, the plant state and the histories are then partial; the next
 * launch is not affected) is read by the next synchronising call.  A block gives up after
 * 1 << 20 polls of a wait (of the order of a second), or after the number of polls in the
 * environment variable MPPI_STEP_SPIN_LIMIT at the time of the call (for tests of this
 * path).  INVAL: x_dev NULL or n_iter outside [0, 1<<20]. */
mppi_status mppi_run_receding_device(mppi_ctx* ctx, float* x_dev, int32_t n_iter, float* u_hist_dev,
                                     float* x_hist_dev);

/* K-shard form, step 1 (Algorithm 2 over samples spread across shards): one iteration of
 * this context's K samples from x0[7] (host) that ends, in place of the update, with the
 * shard's merged partial in row_dev (device, [2 + 2T] floats, written by the launch):
 *   row_dev[0] = rho_g = min_k S_k,  row_dev[1] = eta_g = sum_k exp(-(S_k - rho_g)/lambda),
 *   row_dev[2 + 2t + i] = N_g[t][i] = sum_k exp(-(S_k - rho_g)/lambda) delta_{k,t,i}
 * (eta_g = 0 when no sample of the shard has a finite cost).  U and the statistics are
 * not changed; the iteration counter advances.  Enqueued, unless costs_out ([K] host
 * floats, nullable) asks for the shard's S_k, which synchronises; row_dev must stay
 * valid until the launch has run.  INVAL: row_dev NULL, a non-finite x0,
 * MPPI_WEIGHTS_CEM.  STATE: map or dynamics not set. */
mppi_status mppi_iterate_partial(mppi_ctx* ctx, const float x0[7], float* row_dev, float* costs_out);

/* K-shard form, step 2: merge the n_rows partial rows of one iteration's shards (device,
 * [n_rows][2 + 2T], e.g. gathered from every shard) exactly as the blocks of one launch
 * are merged (rho = min_g rho_g, eta~ = sum_g exp(-(rho_g - rho)/lambda) eta_g,
 * Delta = sum_g exp(-(rho_g - rho)/lambda) N_g / eta~), then smooth and update U and the
 * statistics as mppi_iterate does.  The iteration counter does not advance.  Enqueued;
 * the status (MPPI_E_NONFINITE when no shard had a finite cost) is read by the next
 * synchronising call.  INVAL: rows_dev NULL or n_rows outside [1, 65536]. */
mppi_status mppi_merge_update(mppi_ctx* ctx, const float* rows_dev, int32_t n_rows);

/* Diagnostics of the most recent iteration (synchronises): rho = min_k S_k,
 * eta~ = sum_k exp(-(S_k - rho)/lambda), and the unsmoothed update
 * Delta_t = sum_k w_k delta_{k,t} ([T][2]).  With MPPI_WEIGHTS_CEM, rho is the largest
 * elite cost and eta the number of elite samples.  Any output pointer may be NULL. */
mppi_status mppi_get_stats(mppi_ctx* ctx, float* rho, float* eta, float* delta_out);

/* The perturbations eps ([K][T][2]) that the device generator draws for
 * iteration `iter` (the generator of the rollout kernels, run on its own).
 * Synchronises. */
mppi_status mppi_get_noise(mppi_ctx* ctx, uint32_t iter, float* eps_out);

/* Iteration counter (the Philox counter's third word) for checkpoint/resume:
 * U (mppi_get_controls / mppi_set_controls), the seed and this counter
 * reproduce the next iteration bit for bit.  The counter lives on the device (every
 * iteration launch reads it and advances it); both calls synchronise. */
mppi_status mppi_get_iteration(mppi_ctx* ctx, uint32_t* iter);
mppi_status mppi_set_iteration(mppi_ctx* ctx, uint32_t iter);

/* Rollout schedule actually used (MPPI_SCHED_LANE, _WAVE, _WIDE or _QUAD). */
mppi_status mppi_get_schedule(const mppi_ctx* ctx, int32_t* schedule);

/* Device time of the iteration kernel, measured with HIP events recorded on the
 * context's stream around every launch once enabled.  times_ms[0] = the rollout
 * kernel (which also forms the weights and updates U in its last block; also the
 * forward launch of mppi_objective), summed since timing was last enabled,
 * counts[0] = launches; times_ms[1] and counts[1]
 * the same for the adjoint rollout kernel of mppi_objective_backward (its two
 * gradient reduction kernels excluded).  The events add stream markers between
 * launches, so measure throughput with timing off.  mppi_get_timing synchronises. */
mppi_status mppi_set_timing(mppi_ctx* ctx, int32_t enable);
mppi_status mppi_get_timing(mppi_ctx* ctx, double times_ms[2], int64_t counts[2]);
/* The individual launch durations (ms) behind mppi_get_timing's times_ms[0], oldest
 * first: up to cap of them into ms_out; *n_out = how many were recorded.
 * Synchronises. */
mppi_status mppi_get_timing_samples(mppi_ctx* ctx, float* ms_out, int32_t cap, int32_t* n_out);

/* Differentiation form.  The free-energy objective of Eq. FreeEnergy estimated with
 * this iteration's K samples,
 *   J = -lambda log((1/K) sum_k exp(-S_k/lambda)) = rho - lambda log(eta~/K),
 * at the context's U and network, with the perturbations of iteration `iter` (the
 * counter is not advanced and U is not changed).  The forward pass stores every
 * sample's full state each `ckpt_every` steps (1..16) for the backward pass.
 * Synchronises.  J_out and costs_out ([K]) may be NULL.  Requires h = 32.
 * INVAL: ckpt_every outside [1, 16], h != 32, explore != 0 or MPPI_WEIGHTS_CEM (the
 * objective is defined over importance samples and Algorithm 2's weights only).
 * NONFINITE: no finite cost. */
mppi_status mppi_objective(mppi_ctx* ctx, const float x0[7], uint32_t iter, int32_t ckpt_every,
                           double* J_out, float* costs_out);

/* Gradient of the last mppi_objective's J with respect to U (dJdU, [T][2]) and the
 * network parameters (dJdtheta, packed like mppi_set_dynamics, 1412 floats), by an
 * adjoint rollout that re-runs each checkpointed segment.  Either output may be NULL.
 * Synchronises.  STATE: no objective evaluated since the last change of U, the
 * network, the map or the last mppi_iterate. */
mppi_status mppi_objective_backward(mppi_ctx* ctx, float* dJdU, float* dJdtheta);

/* Allocation-free form of mppi_iterate_device, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It needs no context and calls no hipMalloc, hipFree or other allocating
 * routine: one MPPI iteration (the same kernels, launch shape and results, bit for bit,
 * as a context with this cfg, cost, map and network whose iteration counter is `iter`)
 * reads the caller's device buffers and keeps everything else -- the per-block partial
 * rows, the arrival counters, the statistics, the crash-decay and smoothing tables, and
 * S or the status when their pointers are NULL -- in one static device array of the
 * library (about 4.3 MiB on each device it runs on, held until the process ends).
 * Arguments: cfg and cost as for mppi_create (cfg->schedule AUTO resolves as in
 * mppi_set_dynamics); map_dev [H][W] row-major floats with the geometry of
 * mppi_set_costmap; dims / params_dev the network as for mppi_set_dynamics (params_dev
 * is read as given, not checked for finiteness); x0_dev [7]; iter the Philox counter's
 * third word; U_dev [T][2] in/out, updated in place; S_dev [K] out (NULL: not returned);
 * status_dev [1] out, 0 or MPPI_E_NONFINITE (NULL: not returned).  Every pointer except
 * cfg, cost and dims is a device pointer on `device`, owned by the caller, and must
 * stay valid until the launch has run.  The launch is enqueued on hip_stream and the call
 * returns; only the first call on a device and a call whose (T, sg_window, sg_order,
 * crash_decay) differs from the previous call's synchronise the device (to load the
 * tables).  Every call on a device shares that device's array: calls whose launches
 * overlap in time (other streams, other host threads) race; calls enqueued on one
 * stream in turn do not.  Errors are reported by mppi_last_error(NULL).
 * INVAL: as mppi_create and mppi_set_dynamics, plus K > 16384, sg_window > 31,
 * weighting MPPI_WEIGHTS_CEM, or a NULL map_dev, dims, params_dev, x0_dev or U_dev. */
mppi_status mppi_iterate_noalloc(const mppi_config* cfg, const mppi_cost* cost, int device, void* hip_stream,
                                 const float* map_dev, int32_t H, int32_t W, float origin_x, float origin_y,
                                 float resolution, const int32_t dims[4], const float* params_dev,
                                 const float* x0_dev, uint32_t iter, float* U_dev, float* S_dev,
                                 int32_t* status_dev);

/* Batched form: n independent MPPI problems (instances) that share one cost map,
 * one cost and one FP32 6-32-32-4 network, each with its own K_i, T_i, x0, U and
 * iteration counter, advanced together by one persistent kernel launch per
 * mppi_batch_iterate (replayed from a HIP graph).  Instance i draws its noise with
 * Philox counter word 4 = cfg->instance + i (cfg->k_base and cfg->k_total must be 0).  cfg->schedule picks the work tiles:
 * MPPI_SCHED_QUAD or AUTO (tiles of 64 samples, matrix-core network) or
 * MPPI_SCHED_LANE (tiles of 256); instance i then reproduces, bit for bit, a
 * single-problem context with K_i, T_i, that instance word and that schedule.
 * cfg->K and cfg->T are ignored.  The first iterate times several launch shapes
 * (grid size and work order) on the real problem and keeps the fastest; U and the
 * counters are restored afterwards and every shape gives the same results.  With a
 * NULL stream the batch creates its own (graph capture needs a non-null stream).  With
 * quad tiles allowed the batch also holds 8 bytes per sample and step of every instance
 * (ceil(K_i/64) 64 T_i pairs of floats) for the tiles' noise.
 * INVAL: n outside [1, 65536], an instance's K/T invalid (as in mppi_config), a
 * precision other than FP32, or a schedule other than AUTO, LANE or QUAD. */
typedef struct mppi_batch mppi_batch;
mppi_status mppi_batch_create(const mppi_config* cfg, const mppi_cost* cost, int32_t n, const int32_t* K,
                              const int32_t* T, int device, void* hip_stream, mppi_batch** out);
void mppi_batch_destroy(mppi_batch* b);
const char* mppi_batch_last_error(const mppi_batch* b);
mppi_status mppi_batch_set_costmap(mppi_batch* b, const float* map, int32_t H, int32_t W, float origin_x,
                                   float origin_y, float resolution);
/* dims must be {6, 32, 32, 4}. */
mppi_status mppi_batch_set_dynamics(mppi_batch* b, const int32_t dims[4], const float* params);
/* Instance i's nominal controls ([T_i][2]); every instance starts at 0. */
mppi_status mppi_batch_set_controls(mppi_batch* b, int32_t i, const float* U);
/* One iteration of every instance from x0 ([n][7], host).  Enqueued. */
mppi_status mppi_batch_iterate(mppi_batch* b, const float* x0);
/* Instance i's controls ([T_i][2]) / costs of its last iteration ([K_i]).  Synchronise. */
mppi_status mppi_batch_get_controls(mppi_batch* b, int32_t i, float* U_out);
mppi_status mppi_batch_get_costs(mppi_batch* b, int32_t i, float* S_out);
/* The schedule the autotuner chose: persistent grid size (blocks that take work
 * items from the launch's queue), work order (0 = by instance, 1 = longest horizon
 * first), its measured time per launch, and the rollout schedule of the tiles
 * (MPPI_SCHED_QUAD: 64 samples per tile, four lanes per sample; MPPI_SCHED_LANE: 256
 * samples, one lane each -- both are tried when the configuration's schedule is
 * MPPI_SCHED_AUTO).  Any output pointer may be NULL. */
mppi_status mppi_batch_get_schedule(mppi_batch* b, int32_t* grid, int32_t* order, double* tuned_us,
                                    int32_t* schedule);
mppi_status mppi_batch_synchronize(mppi_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* MPPI_H */
