"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same
seeded inputs.

Bars (FP32 GPU vs FP64 oracle):
  * eps: bit-identical (both sides implement the same counter-based generator).
  * S_k: |S_gpu - S_match| <= 1e-5 * max(|S_match|, 1) for every sample, S_match being the
    oracle's cost with each impulse term that its trajectory decides within 1e-4 of the
    threshold on the side the GPU's cost matches (parity_checks.match_costs).
  * U, stage-isolated: the oracle's FP64 weights/update applied to the GPU's own S and
    the bit-identical eps reproduces the GPU's U within 1e-5 absolute.
  * U, end to end: GPU U vs the oracle's update from S_match, within 1e-5 absolute or
    the rigorous bound the measured cost differences imply; every value is recorded.
"""
import math
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

import parity_checks as pc
from parity_checks import COST_RTOL, U_ATOL, check_iteration as _check_iteration, deltas


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1707_02342_amd import mppi
    mppi.lib()
    return mppi


def _ctrl(M, prob, cmap, params, schedule=0):
    return M.Controller(prob, cmap, params, schedule=schedule)


def _orc(orc, prob, cmap, params):
    return orc.OracleProblem(prob, cmap, params)


def _say(*a):
    print(*a, flush=True)


def _schedules():
    return [1, 2, 3, 4]


# ---------------------------------------------------------------------------
# Noise
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,instance,it", [(0, 0, 0), (0, 0, 7), (0x1234567890AB, 3, 11), (2**64 - 1, 2**32 - 1, 2**32 - 1)])
def test_noise_bit_identical(M, orc, seed, instance, it):
    prob = synth.with_(synth.c1_problem(), K=300, T=37, seed=seed, instance=instance, sigma2=(0.3, 0.35))
    _say("noise", seed, instance, it)
    with _ctrl(M, prob, synth.ring_map(), synth.mlp_params(32, 0)) as c:
        g = c.noise(it)
    r = orc.noise(_orc(orc, prob, synth.ring_map(), synth.mlp_params(32, 0)), it)
    assert g.dtype == r.dtype == np.float32
    mism = np.count_nonzero(g.view(np.uint32) != r.view(np.uint32))
    assert mism == 0, f"{mism} of {g.size} draws differ; max |diff| {np.abs(g - r).max()}"


def test_noise_full_size_bit_identical(M, orc):
    prob = synth.c2_problem(seed=3)
    with _ctrl(M, prob, synth.ring_map(), synth.mlp_params(32, 0)) as c:
        g = c.noise(5)
    r = orc.noise(_orc(orc, prob, synth.ring_map(), synth.mlp_params(32, 0)), 5)
    assert np.array_equal(g.view(np.uint32), r.view(np.uint32))


# ---------------------------------------------------------------------------
# One iteration
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("schedule", _schedules())
@pytest.mark.parametrize("seed", [0, 1])
def test_plain_workload_iteration(M, orc, schedule, seed):
    """K=256, T=30, ring map, cost 100 h + (v_x - 6)^2, lambda = 1, SGF off."""
    prob = synth.c1_problem(seed=seed)
    _say("plain", schedule, seed)
    _check_iteration(M, orc, prob, synth.ring_map(), synth.mlp_params(32, 0), synth.C1_X0,
                     np.zeros((prob.T, 2), np.float32), schedule)


@pytest.mark.parametrize("schedule", _schedules())
def test_plain_workload_warm_controls(M, orc, schedule):
    prob = synth.c1_problem(seed=4)
    _check_iteration(M, orc, prob, synth.ring_map(), synth.mlp_params(32, 0), synth.C1_X0,
                     synth.random_controls(prob.T, 2), schedule, it=3)


@pytest.mark.parametrize("schedule", _schedules())
@pytest.mark.parametrize("K,T", [(1, 1), (1, 30), (7, 5), (63, 17), (65, 31), (257, 9), (1000, 64)])
def test_ragged_shapes(M, orc, schedule, K, T):
    prob = synth.with_(synth.c1_problem(seed=K + T), K=K, T=T)
    _say("ragged", schedule, K, T)
    _check_iteration(M, orc, prob, synth.ring_map(), synth.mlp_params(32, 0), synth.C1_X0,
                     synth.random_controls(T, K), schedule)


@pytest.mark.parametrize("schedule,K", [(2, 2049), (2, 4100), (2, 32768), (3, 2049), (3, 4100), (4, 16385),
                                        (4, 70000), (1, 65537), (1, 70000)])
def test_many_blocks(M, orc, schedule, K):
    """Launches of more than 256 blocks: the partial rows are merged in groups of
    ceil(sqrt(G)) blocks (wave and wide: 8 samples per block, quad: 64, lane: 256)."""
    T = 12
    prob = synth.with_(synth.c1_problem(seed=K), K=K, T=T)
    _say("many blocks", schedule, K)
    _check_iteration(M, orc, prob, synth.ring_map(), synth.mlp_params(32, 0), synth.C1_X0,
                     synth.random_controls(T, 5), schedule)


@pytest.mark.parametrize("schedule", _schedules())
def test_sgf_and_impulses_small(M, orc, schedule):
    """The paper-shaped cost (impulses, slip) with window-9 smoothing on a small K."""
    prob = synth.with_(synth.c2_problem(seed=2), K=512, T=60)
    _check_iteration(M, orc, prob, synth.ellipse_map(), synth.mlp_params(32, 0), synth.C2_X0,
                     synth.random_controls(60, 7, scale=0.2), schedule, impulses=True)


@pytest.mark.parametrize("schedule", _schedules())
@pytest.mark.parametrize("T", [129, 256])
def test_long_horizons_to_the_maximum(M, orc, schedule, T):
    """Horizons past 128 steps up to MPPI_T_MAX (the wave schedule's 8-chunk variant): more
    than 256 controls, so each merging thread also merges a second column and the final
    stage smooths and updates a second control per thread.  Over 129-256 steps a few
    percent of the trajectories pass within 1e-4 of an impulse threshold; each such term
    may take either side (parity_checks.match_costs), every sample is compared."""
    assert T <= M.MPPI_T_MAX
    prob = synth.with_(synth.c2_problem(seed=T), K=300, T=T)
    _say("long horizon", schedule, T)
    _check_iteration(M, orc, prob, synth.ellipse_map(), synth.mlp_params(32, 0), synth.C2_X0,
                     synth.random_controls(T, 11, scale=0.2), schedule, impulses=True)


@pytest.mark.parametrize("schedule", _schedules())
def test_paper_shaped_full_iteration(M, orc, schedule):
    """K=1920, T=100, 2048^2 elliptical map, SGF window 9 (the benchmark's configuration)."""
    prob = synth.c2_problem(seed=0)
    _check_iteration(M, orc, prob, synth.ellipse_map(), synth.mlp_params(32, 0), synth.C2_X0,
                     np.zeros((100, 2), np.float32), schedule, impulses=True)


@pytest.mark.parametrize("schedule", _schedules())
def test_hidden64_fp32(M, orc, schedule):
    if schedule in (2, 3):
        pytest.skip("the wave and wide schedules are h = 32 only")
    prob = synth.with_(synth.c3_problem(K=1024), T=40)
    _check_iteration(M, orc, prob, synth.ring_map(), synth.mlp_params(64, 0), synth.C1_X0,
                     synth.random_controls(40, 9), schedule)


# ---------------------------------------------------------------------------
# Exploration samples (zero-mean samples k >= (1 - alpha) K) and decoupled gamma
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("schedule", _schedules())
@pytest.mark.parametrize("seed", [0, 1])
def test_exploration_paper_parameters(M, orc, schedule, seed):
    """The parameter table's lambda = 12.5, gamma = 0.1, Sigma = Diag(0.0306, 0.0506) with
    alpha = 0.01 (19 of 1920 samples around zero) on the paper-shaped workload; the
    boundary sample 1901 falls inside a block and a sample group of every schedule."""
    prob = synth.explore_problem(seed)
    _say("explore paper", schedule, seed)
    _check_iteration(M, orc, prob, synth.ellipse_map(), synth.mlp_params(32, 0), synth.C2_X0,
                     synth.random_controls(100, 20 + seed, scale=0.2), schedule, it=seed,
                     impulses=True)


@pytest.mark.parametrize("schedule", _schedules())
@pytest.mark.parametrize("K,T,alpha", [(257, 33, 0.25), (100, 20, 1.0), (65, 7, 0.5 / 65),
                                       (4100, 12, 0.3)])
def test_exploration_fractions(M, orc, schedule, K, T, alpha):
    prob = synth.with_(synth.c1_problem(seed=K), K=K, T=T, gamma=0.5, explore=alpha)
    _say("explore", schedule, K, T, alpha)
    _check_iteration(M, orc, prob, synth.ring_map(), synth.mlp_params(32, 0), synth.C1_X0,
                     synth.random_controls(T, 3, scale=0.5), schedule)


@pytest.mark.parametrize("schedule", [1, 4])
def test_exploration_hidden64(M, orc, schedule):
    """h = 64 FP32 on the lane and quad schedules with exploration samples."""
    prob = synth.with_(synth.c3_problem(K=1024), T=40, gamma=0.3, explore=0.05)
    _check_iteration(M, orc, prob, synth.ring_map(), synth.mlp_params(64, 0), synth.C1_X0,
                     synth.random_controls(40, 9), schedule)


def test_exploration_rejected_outside_unit_interval(M):
    for alpha in (-0.1, 1.5, float("nan")):
        prob = synth.with_(synth.c1_problem(), explore=alpha)
        with pytest.raises(M.MppiError):
            M.Controller(prob, synth.ring_map(), synth.mlp_params(32, 0))


def test_objective_rejects_exploration(M):
    prob = synth.with_(synth.c5_problem(), K=256, T=20, explore=0.1)
    with M.Controller(prob, synth.ring_map(), synth.mlp_params(32, 0)) as c:
        with pytest.raises(M.MppiError):
            c.objective(synth.C1_X0, 0)


# ---------------------------------------------------------------------------
# Receding horizon (Algorithm 1's outer loop)
# ---------------------------------------------------------------------------

def test_receding_horizon_loop(M, orc):
    """Warm-started receding-horizon loop on the paper-shaped workload: every tenth
    iteration's costs and U checked against the oracle from the same (x0, U) inputs
    (cost bar, end-to-end U within 1e-5 or its measured-difference bound, recorded),
    plant steps checked, and the device-resident loop reproduces the host-driven one bit
    for bit."""
    prob = synth.c2_problem(seed=1)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    op = _orc(orc, prob, cmap, params)
    n = 100
    x = synth.C2_X0.copy()
    us, xs = [], [x.copy()]
    worst_u, worst_x = 0.0, 0.0
    with _ctrl(M, prob, cmap, params) as c:
        for i in range(n):
            U_in = c.controls()
            S_g, _ = c.iterate(x, want_costs=True)
            U_out = c.controls()
            if i % 10 == 0 or i == n - 1:
                ref = orc.iterate(op, x, U_in, i)
                eps = orc.noise(op, i)
                S_match, err, info = pc.check_costs(orc, op, prob, cmap, params, x, U_in, eps, S_g, ref.S,
                                                    True, 0.0)
                st2, w, rho, eta = orc.weights(S_g.astype(np.float64), prob.lam)
                Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
                U_iso = U_in.astype(np.float64) + Mx @ np.tensordot(w, deltas(prob, eps, U_in), axes=(0, 0))
                e_iso = float(np.abs(U_out - U_iso).max())
                assert e_iso <= U_ATOL
                e2e, _ = pc.end_to_end(orc, prob, S_g, S_match, eps, U_in, U_out, e_iso, "IT-receding",
                                       step=i, **info)
                worst_u = max(worst_u, e2e)
            u0 = c.shift()
            np.testing.assert_array_equal(u0, U_out[0])
            x_next = c.plant_step(x, u0)
            xr = orc.plant_step(op, x.astype(np.float64), u0.astype(np.float64))
            worst_x = max(worst_x, np.max(np.abs(x_next - xr) / np.maximum(np.abs(xr), 1.0)))
            x = x_next
            us.append(u0)
            xs.append(x.copy())
    _say(f"receding: worst end-to-end |dU| {worst_u:.2e}, worst plant rel {worst_x:.2e}")
    assert worst_x <= 1e-5
    with _ctrl(M, prob, cmap, params) as c:
        uh, xh, st = M.mppi_run_receding(c.ctx, synth.C2_X0, n)
    assert np.array_equal(uh, np.array(us))
    assert np.array_equal(xh, np.array(xs))


@pytest.mark.parametrize("seed", range(10))
def test_paper_shaped_receding_seeds(M, orc, seed):
    """The benchmark's workload for every Philox seed 0-9: 100 warm-started receding
    steps (iterate, shift, plant step) with the automatic schedule; the iterations at
    steps 0, 33, 66 and 99 are checked against the oracle from that step's own state,
    controls and counter (cost bar, stage-isolated and end-to-end U, recorded), and the
    device-resident loop reproduces the host loop bit for bit."""
    prob = synth.c2_problem(seed=seed)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    op = _orc(orc, prob, cmap, params)
    n = 100
    x = synth.C2_X0.copy()
    us, xs = [], [x.copy()]
    _say("paper-shaped receding seed", seed)
    with _ctrl(M, prob, cmap, params) as c:
        for i in range(n):
            U_in = c.controls()
            S_g, _ = c.iterate(x, want_costs=True)
            U_out = c.controls()
            if i in (0, 33, 66, 99):
                ref = orc.iterate(op, x, U_in, i)
                eps = orc.noise(op, i)
                S_match, err, info = pc.check_costs(orc, op, prob, cmap, params, x, U_in, eps, S_g, ref.S,
                                                    True, 0.0)
                st2, w, rho, eta = orc.weights(S_g.astype(np.float64), prob.lam)
                Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
                U_iso = U_in.astype(np.float64) + Mx @ np.tensordot(w, deltas(prob, eps, U_in), axes=(0, 0))
                e_iso = float(np.abs(U_out - U_iso).max())
                assert e_iso <= U_ATOL, f"step {i}: stage-isolated |dU| {e_iso:.3e}"
                pc.end_to_end(orc, prob, S_g, S_match, eps, U_in, U_out, e_iso, "IT-paper-seed",
                              seed=seed, step=i, schedule=c.schedule, **info)
            u0 = c.shift()
            x = c.plant_step(x, u0)
            us.append(u0)
            xs.append(x.copy())
    with _ctrl(M, prob, cmap, params) as c:
        uh, xh, st = M.mppi_run_receding(c.ctx, synth.C2_X0, n)
    assert np.array_equal(uh, np.array(us)) and np.array_equal(xh, np.array(xs))


@pytest.mark.parametrize("schedule", _schedules())
def test_step_device_matches_receding_loop(M, schedule):
    """mppi_step_device (iterate, shift and plant step in one launch, on device data)
    reproduces mppi_run_receding bit for bit, and advances the device-side counter."""
    import torch
    prob = synth.with_(synth.c2_problem(seed=3), K=700, T=40)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    n = 12
    with _ctrl(M, prob, cmap, params, schedule) as c:
        uh, xh, _ = M.mppi_run_receding(c.ctx, synth.C2_X0, n)
        U_ref = c.controls()
    stream = torch.cuda.current_stream()
    with M.Controller(prob, cmap, params, stream=int(stream.cuda_stream), schedule=schedule) as c:
        x = torch.tensor(synth.C2_X0, device="cuda")
        u0 = torch.zeros(2, device="cuda")
        us = []
        for i in range(n):
            M.mppi_step_device(c.ctx, x.data_ptr(), u0.data_ptr())
            us.append(u0.cpu().numpy().copy())
        torch.cuda.synchronize()
        assert np.array_equal(np.array(us), uh)
        assert np.array_equal(x.cpu().numpy(), xh[-1])
        assert np.array_equal(c.controls(), U_ref)
        assert c.iteration == n


def test_step_device_graph_replay(M):
    """One receding-horizon step captured in a HIP graph and replayed: every replay,
    with eager work and synchronisations in between, equals the eager step sequence."""
    import torch
    prob = synth.with_(synth.c2_problem(seed=4), K=1920, T=100)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    n = 6
    s = torch.cuda.Stream()
    with M.Controller(prob, cmap, params, stream=int(s.cuda_stream)) as ref:
        xr = torch.tensor(synth.C2_X0, device="cuda")
        ur = torch.zeros(2, device="cuda")
        ref_x, ref_u, ref_U = [], [], []
        for i in range(n + 1):
            with torch.cuda.stream(s):
                M.mppi_step_device(ref.ctx, xr.data_ptr(), ur.data_ptr())
            s.synchronize()
            ref_x.append(xr.cpu().numpy().copy())
            ref_u.append(ur.cpu().numpy().copy())
            ref_U.append(ref.controls())
    with M.Controller(prob, cmap, params, stream=int(s.cuda_stream)) as c:
        x = torch.tensor(synth.C2_X0, device="cuda")
        u0 = torch.zeros(2, device="cuda")
        # the first step eagerly (the graph is captured from the second on)
        with torch.cuda.stream(s):
            M.mppi_step_device(c.ctx, x.data_ptr(), u0.data_ptr())
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            M.mppi_step_device(c.ctx, x.data_ptr(), u0.data_ptr())
        # capture does not run the step: the state is still the eager step's
        s.synchronize()
        assert np.array_equal(x.cpu().numpy(), ref_x[0])
        for i in range(1, n + 1):
            g.replay()
            torch.cuda.synchronize()
            junk = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
            assert junk == 1000.0
            assert np.array_equal(x.cpu().numpy(), ref_x[i]), f"replay {i}: state"
            assert np.array_equal(u0.cpu().numpy(), ref_u[i]), f"replay {i}: u0"
            assert np.array_equal(c.controls(), ref_U[i]), f"replay {i}: U"
        assert c.iteration == n + 1


def test_timing_samples(M):
    prob = synth.c1_problem(seed=0)
    with _ctrl(M, prob, synth.ring_map(), synth.mlp_params(32, 0)) as c:
        M.mppi_set_timing(c.ctx, True)
        for _ in range(7):
            c.iterate(synth.C1_X0)
        samples = M.mppi_get_timing_samples(c.ctx)
        (t, _), (n, _) = M.mppi_get_timing(c.ctx)
    assert len(samples) == 7 == n
    assert np.all(samples > 0)
    assert abs(samples.sum() - t) <= 1e-3 * t


# ---------------------------------------------------------------------------
# Determinism, resume, error paths
# ---------------------------------------------------------------------------

def test_bitwise_deterministic_and_resume(M, orc):
    prob = synth.c2_problem(seed=5)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    outs = []
    for _ in range(2):
        with _ctrl(M, prob, cmap, params) as c:
            for i in range(3):
                c.iterate(synth.C2_X0)
            outs.append(c.controls())
            it = c.iteration
    assert np.array_equal(outs[0], outs[1])
    with _ctrl(M, prob, cmap, params) as c:
        for i in range(2):
            c.iterate(synth.C2_X0)
        U2 = c.controls()
    with _ctrl(M, prob, cmap, params) as c:
        c.set_controls(U2)
        c.iteration = 2
        c.iterate(synth.C2_X0)
        assert np.array_equal(c.controls(), outs[0])
        assert c.iteration == it


def test_all_nonfinite_leaves_controls(M, orc):
    prob = synth.with_(synth.c1_problem(), K=64, T=10)
    nan_map = synth.constant_map(float("nan"))
    U0 = synth.random_controls(10, 1)
    with _ctrl(M, prob, nan_map, synth.mlp_params(32, 0)) as c:
        c.set_controls(U0)
        S, st = c.iterate(synth.C1_X0, want_costs=True)
        assert st == M.MPPI_E_NONFINITE
        assert np.all(np.isinf(S))
        U, st2 = M.mppi_get_controls(c.ctx, 10)
        assert st2 == M.MPPI_E_NONFINITE
        assert np.array_equal(U, U0)


def test_partial_nonfinite_samples_get_zero_weight(M, orc):
    """A map that is NaN beyond a column boundary: samples that reach it get S = inf and
    weight 0.  The boundary is put in a wide gap between the samples' largest x values
    near their median, so about half of the samples touch it and none is close to it."""
    prob = synth.with_(synth.c1_problem(seed=3), K=256, T=30)
    params = synth.mlp_params(32, 0)
    x0 = np.array([20.8, 12.8, 0.0, 0.0, 6.0, 0.0, 0.0], np.float32)
    op = _orc(orc, prob, synth.ring_map(), params)
    _, tr = orc.rollout(op, x0, np.zeros((30, 2), np.float32), orc.noise(op, 0), traj=True)
    cmap, gap = synth.split_nan_map(tr[:, :, 0].max(axis=1), 12.8)
    assert gap > 1e-4, gap
    S, U = _check_iteration(M, orc, prob, cmap, params, x0, np.zeros((30, 2), np.float32), 1)
    assert np.isinf(S).any() and np.isfinite(S).any()


def test_state_errors(M):
    prob = synth.c1_problem()
    ctx = M.mppi_create(M.make_config(prob), M.make_cost(prob.cost), 0, M.current_stream())
    try:
        with pytest.raises(M.MppiError) as e:
            M.mppi_iterate(ctx, synth.C1_X0)
        assert e.value.status == M.MPPI_E_STATE
        with pytest.raises(M.MppiError):
            M.mppi_set_dynamics(ctx, 48, np.zeros(10, np.float32))
        bad = synth.mlp_params(32, 0).copy()
        bad[5] = np.nan
        with pytest.raises(M.MppiError):
            M.mppi_set_dynamics(ctx, 32, bad)
        with pytest.raises(M.MppiError):
            M.mppi_set_costmap(ctx, np.zeros((1, 5), np.float32), 0.0, 0.0, 0.1)
        x = synth.C1_X0.copy()
        x[2] = np.inf
        M.mppi_set_costmap(ctx, synth.ring_map().data, 0.0, 0.0, 0.1)
        M.mppi_set_dynamics(ctx, 32, synth.mlp_params(32, 0))
        with pytest.raises(M.MppiError):
            M.mppi_iterate(ctx, x)
    finally:
        M.mppi_destroy(ctx)
