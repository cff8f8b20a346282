"""GPU parity of Algorithm 3 (cross-entropy weights): the HIP path through the C ABI
against the CPU oracle on the same seeded inputs, for every schedule.

Bars:
  * S_k as for Algorithm 2 (<= 1e-5 relative against the FP64 oracle; impulse costs
    within 1e-4 of a threshold excluded).
  * Stage-isolated (hard gate): the oracle's elite selection applied to the GPU's own
    FP32 costs picks the set whose delta average reproduces the GPU's U within 1e-5, and
    the GPU's statistics (largest elite cost, elite count) match it exactly.
  * End to end: the elite set from the FP64 costs differs from the GPU's only in samples
    whose costs lie within 1e-5 (relative) of the elite threshold, and the difference in U
    is exactly that swap, averaged and smoothed (within 1e-5).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

COST_RTOL = 1e-5
U_ATOL = 1e-5


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1707_02342_amd import mppi
    mppi.lib()
    return mppi


def _say(*a):
    print(*a, flush=True)


def _deltas(prob, eps, U0):
    d = eps.astype(np.float64).copy()
    alpha = float(np.float32(prob.explore))
    zero_mean = ~(np.arange(d.shape[0]) < (1.0 - alpha) * d.shape[0])
    d[zero_mean] -= U0.astype(np.float64)[None]
    return d


def _check_cem(M, orc, prob, cmap, params, x0, U0, schedule, it=0, impulses=False):
    with M.Controller(prob, cmap, params, schedule=schedule) as c:
        c.set_controls(U0)
        c.iteration = it
        S, st = c.iterate(x0, want_costs=True)
        Ug = c.controls()
        z_g, n_g, delta_g = c.stats()
    op = orc.OracleProblem(prob, cmap, params)
    eps = orc.noise(op, it)
    ref = orc.iterate(op, x0, U0, it)
    zeta = orc.cem_zeta(prob.K, prob.elite)
    assert st == M.MPPI_OK and ref.status == orc.OK
    fin = np.isfinite(ref.S)
    assert np.array_equal(np.isfinite(S), fin), "non-finite samples differ"
    Sf, Rf = np.where(fin, S.astype(np.float64), 0.0), np.where(fin, ref.S, 0.0)
    err = np.abs(Sf - Rf) / np.maximum(np.abs(Rf), 1.0)
    if impulses:
        margin = orc.threshold_margins(op, x0, U0, eps)
        near = margin < 1e-4
        assert near.mean() < 1e-3
        err = np.where(near, 0.0, err)
    assert err.max() <= COST_RTOL, f"max rel dS {err.max():.3e}"
    d = _deltas(prob, eps, U0)
    Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
    # stage-isolated: the oracle's Algorithm 3 on the GPU's costs
    st2, w_iso, z_iso, n_iso = orc.weights_cem(S.astype(np.float64), zeta)
    delta_iso = np.tensordot(w_iso, d, axes=(0, 0))
    e_iso = np.abs(Ug - (U0.astype(np.float64) + Mx @ delta_iso)).max()
    assert e_iso <= U_ATOL, f"stage-isolated |dU| {e_iso:.3e}"
    np.testing.assert_allclose(delta_g, delta_iso, rtol=0, atol=1e-6)
    assert n_g == n_iso and z_g == np.float32(z_iso), (n_g, n_iso, z_g, z_iso)
    # end to end: the two elite sets differ only at the threshold, and U by that swap
    E_g, E_r = set(np.nonzero(w_iso)[0]), set(np.nonzero(ref.w)[0])
    swapped = sorted(E_g ^ E_r)
    z_r = ref.rho
    for k in swapped:
        assert abs(ref.S[k] - z_r) <= 1e-5 * max(abs(z_r), 1.0), (k, ref.S[k], z_r)
    pred = Mx @ ((d[sorted(E_g - E_r)].sum(axis=0) - d[sorted(E_r - E_g)].sum(axis=0)) / n_iso) if swapped else 0.0
    resid = np.abs(Ug - ref.U - pred).max()
    _say(f"CEM K={prob.K} T={prob.T} sched={schedule} zeta={zeta}: rel dS {err.max():.2e}, |dU| iso "
         f"{e_iso:.2e}, swapped {len(swapped)}, e2e residual {resid:.2e}")
    assert resid <= U_ATOL
    return S, Ug


def _schedules():
    return [1, 2, 3, 4]


@pytest.mark.parametrize("schedule", _schedules())
@pytest.mark.parametrize("seed", [0, 1])
def test_cem_paper_parameters(M, orc, schedule, seed):
    """K=1920, T=100, the parameter table's lambda, gamma, Sigma and eliteness
    threshold 0.8 (384 elite samples), 2048^2 elliptical map, SGF window 9."""
    prob = synth.cem_problem(seed)
    _say("cem paper", schedule, seed)
    _check_cem(M, orc, prob, synth.ellipse_map(), synth.mlp_params(32, 0), synth.C2_X0,
               synth.random_controls(100, 30 + seed, scale=0.2), schedule, it=seed, impulses=True)


@pytest.mark.parametrize("schedule", _schedules())
@pytest.mark.parametrize("K,T,elite", [(1, 1, 0.0), (7, 5, 0.5), (65, 31, 0.9), (257, 9, 0.0),
                                       (1000, 64, 0.8), (4100, 12, 0.95), (300, 200, 0.8),
                                       (50, 256, 0.5), (9000, 10, 0.3)])
def test_cem_ragged(M, orc, schedule, K, T, elite):
    prob = synth.with_(synth.c1_problem(seed=K + T), K=K, T=T, weighting=1, elite=elite)
    _say("cem ragged", schedule, K, T, elite)
    _check_cem(M, orc, prob, synth.ring_map(), synth.mlp_params(32, 0), synth.C1_X0,
               synth.random_controls(T, K), schedule)


@pytest.mark.parametrize("schedule,K", [(2, 32768), (4, 70000), (1, 70000)])
def test_cem_many_blocks(M, orc, schedule, K):
    prob = synth.with_(synth.c1_problem(seed=K), K=K, T=12, weighting=1, elite=0.8)
    _check_cem(M, orc, prob, synth.ring_map(), synth.mlp_params(32, 0), synth.C1_X0,
               synth.random_controls(12, 5), schedule)


@pytest.mark.parametrize("schedule", _schedules())
def test_cem_with_exploration(M, orc, schedule):
    prob = synth.with_(synth.cem_problem(2), K=700, T=60, explore=0.05)
    _check_cem(M, orc, prob, synth.ellipse_map(), synth.mlp_params(32, 0), synth.C2_X0,
               synth.random_controls(60, 8, scale=0.2), schedule, impulses=True)


@pytest.mark.parametrize("schedule", _schedules())
def test_cem_all_costs_tied(M, orc, schedule):
    """No cost terms at all: every S_k = 0, so the elite set is the zeta lowest sample
    indices and the update is the plain average of their perturbations."""
    cost = synth.CostParams(w_map=0.0, w_speed=0.0, w_slip=0.0)
    prob = synth.with_(synth.c1_problem(seed=9), K=300, T=16, gamma=0.0, weighting=1, elite=0.7,
                       cost=cost)
    U0 = synth.random_controls(16, 9)
    with M.Controller(prob, synth.ring_map(), synth.mlp_params(32, 0), schedule=schedule) as c:
        c.set_controls(U0)
        S, st = c.iterate(synth.C1_X0, want_costs=True)
        Ug = c.controls()
        z, n, _ = c.stats()
    assert st == M.MPPI_OK and not S.any() and n == 90 and z == 0.0
    op = orc.OracleProblem(prob, synth.ring_map(), synth.mlp_params(32, 0))
    eps = orc.noise(op, 0).astype(np.float64)
    np.testing.assert_allclose(Ug, U0 + eps[:90].mean(axis=0), rtol=0, atol=1e-6)


@pytest.mark.parametrize("schedule", _schedules())
def test_cem_nonfinite_samples(M, orc, schedule):
    """A map that is NaN beyond a column boundary that about half of the samples cross
    (placed in a wide gap of their largest x): those get S = inf and are never elite.
    With every sample non-finite the status is NONFINITE and U is unchanged."""
    prob = synth.with_(synth.c1_problem(seed=3), K=256, T=30, weighting=1, elite=0.8)
    params = synth.mlp_params(32, 0)
    x0 = np.array([20.8, 12.8, 0.0, 0.0, 6.0, 0.0, 0.0], np.float32)
    U0 = np.zeros((30, 2), np.float32)
    op = orc.OracleProblem(prob, synth.ring_map(), params)
    _, tr = orc.rollout(op, x0, U0, orc.noise(op, 0), traj=True)
    cmap, gap = synth.split_nan_map(tr[:, :, 0].max(axis=1), 12.8)
    assert gap > 1e-4, gap
    S, _ = _check_cem(M, orc, prob, cmap, params, x0, U0, schedule)
    n_inf = int(np.isinf(S).sum())
    assert 0 < n_inf < 256
    _say("non-finite samples:", n_inf)
    nan_map = synth.constant_map(float("nan"))
    U1 = synth.random_controls(30, 4)
    with M.Controller(prob, nan_map, params, schedule=schedule) as c:
        c.set_controls(U1)
        S, st = c.iterate(synth.C1_X0, want_costs=True)
        assert st == M.MPPI_E_NONFINITE and np.all(np.isinf(S))
        np.testing.assert_array_equal(c.controls(), U1)


@pytest.mark.parametrize("schedule", _schedules())
def test_cem_receding_device_loop_matches_host_loop(M, schedule):
    """mppi_run_receding (iteration, shift and plant step in one launch each) equals the
    host-driven loop of mppi_iterate, mppi_shift and mppi_plant_step bit for bit."""
    prob = synth.with_(synth.cem_problem(5), K=640, T=50)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    n = 10
    with M.Controller(prob, cmap, params, schedule=schedule) as c:
        uh, xh, _ = M.mppi_run_receding(c.ctx, synth.C2_X0, n)
    with M.Controller(prob, cmap, params, schedule=schedule) as c:
        x = synth.C2_X0.copy()
        for i in range(n):
            c.iterate(x)
            u0 = c.shift()
            assert np.array_equal(u0, uh[i])
            x = c.plant_step(x, u0)
            assert np.array_equal(x, xh[i + 1])


def test_cem_rejections(M):
    base = synth.with_(synth.c1_problem(), weighting=1)
    for bad in (dict(elite=1.0), dict(elite=-0.1), dict(elite=float("nan")), dict(elite=0.999, K=100),
                dict(weighting=2)):
        with pytest.raises(M.MppiError):
            M.Controller(synth.with_(base, **bad), synth.ring_map(), synth.mlp_params(32, 0))
    with M.Controller(synth.with_(synth.c5_problem(), K=256, T=20, weighting=1), synth.ring_map(),
                      synth.mlp_params(32, 0)) as c:
        with pytest.raises(M.MppiError):
            c.objective(synth.C1_X0, 0)
    with pytest.raises(M.MppiError):
        M.Batch(synth.cem_problem(0), [256, 300], [20, 30], synth.ellipse_map(), synth.mlp_params(32, 0))
