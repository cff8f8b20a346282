// Kernel argument blocks shared by the host runtime and the HIP kernels.
// Passed by value as kernel arguments (no constant-memory uploads per call).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mppi {

constexpr int kStateDim = 7;

// Multi-step receding launch: the words its blocks signal each other through (a device
// buffer of kSyncWords(G) words per context, zero when the context is created).  Every
// word holds a step number, step_base + s + 1 for step s of a launch, which grows over
// the context's multi-step launches, so no word is ever reset.
//   copy c < kSignalCopies of group word g: the last step whose group row g is out (the
//     copies kSignalSpacing words, 4 KiB, apart; rollout block b polls copy
//     b mod kSignalCopies, so that not every block polls the same memory);
//   arrival word b (at kArriveOffset + b, b < G): the last step whose row of rollout
//     block b is out.
constexpr int kSignalCopies = 16;
constexpr int kSignalSpacing = 1024;
constexpr int kArriveOffset = kSignalCopies * kSignalSpacing;
constexpr inline int kSyncWords(int G) { return kArriveOffset + G; }
constexpr int kCtrlDim = 2;
constexpr int kNetIn = 6;
constexpr int kNetOut = 4;
constexpr int kTMax = 256;

// The per-block partial rows of one launch (G blocks) are merged in two levels:
// groups of merge_group_size(G) consecutive blocks, then the merge_groups(G) group
// rows.  16 up to 256 blocks, ceil(sqrt(G)) beyond, so neither level grows faster
// than sqrt(G).
__host__ __device__ constexpr inline int merge_group_size(int G) {
  int s = 16;
  while (s * s < G) ++s;
  return s;
}
__host__ __device__ constexpr inline int merge_groups(int G) {
  const int s = merge_group_size(G);
  return (G + s - 1) / s;
}

// Philox key and counter words that are fixed within one iteration, plus the
// noise standard deviations sqrt(Sigma_ii) (FP32, correctly rounded on the host).
struct NoiseKey {
  uint32_t key_lo, key_hi;   // seed words
  uint32_t iter;             // third counter word
  uint32_t instance;         // fourth counter word
  float sig0, sig1;
  uint32_t k_base;           // global index of sample 0 (second counter word = k_base + k)
};

// Cost map geometry and state-cost weights.
struct CostArgs {
  int H, W;
  float ox, oy, res;
  float w_map, w_speed, w_slip, v_des;
  float crash_cost, map_thresh, slip_cost, slip_thresh;
};

// One rollout launch: K samples, T steps, from x0 (by value, or read from x0_dev).
// Dynamics models: the 6-h-h-4 tanh network, or the basis-function model.
constexpr int kModelNet = 0;
constexpr int kModelBasis = 1;
constexpr int kModelAny = -1;   // a kernel that serves either model (chosen by RolloutArgs::model)

struct RolloutArgs {
  const float* U;          // [T][2] nominal controls
  const float* map;        // [H][W]
  const float* params;     // packed network parameters (FP32)
  const float* decay;      // [T+1] fl32(crash_decay^t)
  const float* x0_dev;     // nullable: read x0 from here instead of x0[]
  float* S;                // [K] trajectory costs
  float* part;             // [G][2 + 2T] per-block (rho_g, eta_g, N_g[T][2])
  float* part2;            // [2][merge_groups(G)][2 + 2T] per-group merges (the second set: multi-step)
  unsigned* cnt;           // [merge_groups(G) + 1] arrival counters, zero between launches
  const float* sg;         // [T][sg_window] smoothing rows (null when window == 1)
  float* Uout;             // [T][2], updated in place by the last block
  float* stats;            // [2 + 2T]: rho, eta~, Delta[T][2]
  int* status;             // 0 or MPPI_E_NONFINITE for this iteration
  int G;                   // rollout blocks of this launch
  int sg_window;
  int update_U;            // 0: weights and Delta only (objective evaluation)
  unsigned* iter_dev;      // nullable: the iteration counter (read at the start of the launch in place
                           // of nk.iter, advanced by the final merge)
  float* ckpt;             // nullable: [K][n_ckpt][8] full states every ckpt_every steps
  int ckpt_every;
  float x0[kStateDim];
  int K, T;
  int K_imp;               // samples k < K_imp are drawn around U (v = u + eps); the rest
                           // are exploration samples around zero (v = eps)
  int cem_zeta;            // 0: Algorithm 2's weights; > 0: Algorithm 3 with this many elite samples
  float* D;                // Algorithm 3 only: [K][T][2] delta rows (v - u) of every sample
  // Quad schedule (nullable): the launch's noise, [tiles][4 waves][T][16][2], written as
  // the rollout draws it and read back by the weighted perturbation sum in place of a
  // second draw (the same values); null: drawn again.
  float* eps_store;
  float dt;
  float inv_lambda;
  float gcs0, gcs1;        // gamma / Sigma_ii (control-cost weights)
  float u_lo0, u_lo1, u_hi0, u_hi1;
  NoiseKey nk;
  CostArgs cost;
  int hidden;              // network width (32 or 64)
  int model;               // kModelNet (params = packed network) or kModelBasis (params = Theta[25][4])
  // Receding-horizon step (recede = 1): after the update the final merge also shifts U
  // (u_0 out, u_{t-1} <- u_t, u_{T-1} <- 0) and advances the plant x <- F(x, g(u_0)) in
  // place in x0_dev.
  int recede;
  float* u0_out;           // nullable: [2] u_0 of this step
  float* x_copy;           // nullable: [7] a copy of the new plant state
  // K-shard form: when set, the final merge writes the launch's merged row
  // (rho, eta, N[T][2]) here ([2 + 2T]) and leaves U, the statistics and the smoothing
  // to a later merge of every shard's row (merge_update_kernel).
  float* row_out;
  // Multi-step receding launch (the split wave kernel, launched cooperatively with G
  // rollout blocks and merge_groups(G) merger blocks): n_steps receding steps in one launch
  // (0 or 1: one step), step s signalled as step_base + s + 1 in the words of sync
  // ([kSyncWords(G)], see kSignalCopies); u0_out and x_copy then point to [n_steps][2]
  // and [n_steps][7] histories (step s writes entry s).
  int n_steps;
  unsigned* sync;
  unsigned step_base;
  unsigned spin_limit;   // polls of one wait before the launch gives up (0: 1 << 20)
};

constexpr int kCkptStride = 8;   // floats per checkpointed state (7 + pad)

// Adjoint of the free-energy objective J = rho - lambda log(eta~/K) through every
// sample's rollout (one launch over all samples).
struct AdjointArgs {
  const float* U;
  const float* map;
  const float* params;
  const float* decay;
  const float* S;          // [K] costs of the forward pass
  const float* stats;      // rho, eta~ of the forward pass
  const float* ckpt;       // [K][n_ckpt][8]
  float* gpart;            // [G][P + 2T] per-block gradient partials
  int K, T, ckpt_every, n_ckpt;
  float dt, inv_lambda;
  float u_lo0, u_lo1, u_hi0, u_hi1;
  NoiseKey nk;
  CostArgs cost;
};

}  // namespace mppi
