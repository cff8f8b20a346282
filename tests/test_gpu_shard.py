"""GPU parity of the K-shard form on one GPU: the samples of one iteration split over
several contexts (global sample indices k_base .. k_base + K_g - 1 of k_total), each
exporting its merged Algorithm 2 partial (rho_g, eta_g, N_g[T][2]) through
mppi_iterate_partial, then one exact merge and update (mppi_merge_update).  This is what
each GPU of a sharded iteration would compute; the rows' all-gather between devices is
not exercised here.

Bars:
  * eps and S: every shard's samples equal the unsharded context's samples of the same
    global index bit for bit (same generator counter, same per-sample arithmetic).
  * rows: rho_g is the shard's minimum cost exactly; eta_g and N_g agree with the FP64
    sums over the shard's own FP32 costs to 1e-5 relative (N_g: of eta_g max|delta|).
  * U: the merged update equals the unsharded iteration's within 1e-6 (the two only
    differ in merge order), and the oracle's full-K iteration to the usual bars
    (stage-isolated 1e-5; end to end 1e-5 or its recorded bound).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

import parity_checks as pc
from parity_checks import U_ATOL, deltas


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1707_02342_amd import mppi
    mppi.lib()
    return mppi, torch


def _say(*a):
    print(*a, flush=True)


def _shards(M, torch, prob, cmap, params, x0, U0, it, sizes, schedule=0):
    """Run the shards of `sizes` (summing to prob.K); returns their S (concatenated),
    rows [n][2 + 2T], and the merged U from two different shard contexts."""
    assert sum(sizes) == prob.K
    T = prob.T
    rows = torch.zeros((len(sizes), 2 + 2 * T), dtype=torch.float32, device="cuda")
    ctls, S_parts, base = [], [], 0
    try:
        for g, k in enumerate(sizes):
            p = synth.with_(prob, K=k, k_base=base, k_total=prob.K)
            c = M.Controller(p, cmap, params, schedule=schedule)
            ctls.append(c)
            c.set_controls(U0)
            c.iteration = it
            S = np.zeros(k, np.float32)
            M.mppi_iterate_partial(c.ctx, x0, rows[g].data_ptr(), S)
            S_parts.append(S)
            base += k
        torch.cuda.synchronize()
        merged = []
        for c in (ctls[0], ctls[-1]):
            M.mppi_merge_update(c.ctx, rows.data_ptr(), len(sizes))
            U, st = M.mppi_get_controls(c.ctx, T)
            assert st == M.MPPI_OK
            merged.append((U, c.stats()))
        eps_last = ctls[-1].noise(it)
        iters = [c.iteration for c in ctls]
    finally:
        for c in ctls:
            c.close()
    assert iters == [it + 1] * len(sizes), "each shard's launch advances its counter once"
    return np.concatenate(S_parts), rows.cpu().numpy(), merged, eps_last


def _check(M, torch, orc, prob, cmap, params, x0, U0, it, sizes, impulses):
    _say(f"shards {sizes} of K={prob.K} T={prob.T} explore={prob.explore} it={it}")
    S_sh, rows, merged, eps_last = _shards(M, torch, prob, cmap, params, x0, U0, it, sizes)
    (U_a, (rho_a, eta_a, D_a)), (U_b, _) = merged
    np.testing.assert_array_equal(U_a, U_b)
    # the unsharded iteration on the same inputs
    with M.Controller(prob, cmap, params) as c:
        c.set_controls(U0)
        c.iteration = it
        S_full, st = c.iterate(x0, want_costs=True)
        U_full = c.controls()
        eps_full = c.noise(it)
    assert st == M.MPPI_OK
    np.testing.assert_array_equal(S_sh, S_full)
    np.testing.assert_array_equal(eps_last, eps_full[prob.K - sizes[-1]:])
    du_full = float(np.abs(U_a - U_full).max())
    _say(f"  merged vs unsharded: max |dU| {du_full:.2e}")
    assert du_full <= 1e-6
    # each row against FP64 sums over the shard's own costs
    d = deltas(prob, orc.noise(orc.OracleProblem(prob, cmap, params), it), U0)
    base = 0
    for g, k in enumerate(sizes):
        S = S_sh[base:base + k].astype(np.float64)
        rho = S.min()
        w = np.exp(-(S - rho) / prob.lam)
        eta = w.sum()
        N = np.tensordot(w, d[base:base + k], axes=(0, 0)).reshape(-1)
        assert rows[g, 0] == np.float32(rho)
        assert abs(rows[g, 1] - eta) <= 1e-5 * eta
        assert np.abs(rows[g, 2:] - N).max() <= 1e-5 * eta * np.abs(d[base:base + k]).max()
        base += k
    # the merged update against the oracle's full-K iteration
    op = orc.OracleProblem(prob, cmap, params)
    eps = orc.noise(op, it)
    ref = orc.iterate(op, x0, U0, it)
    assert ref.status == orc.OK
    S_match, err, info = pc.check_costs(orc, op, prob, cmap, params, x0, U0, eps, S_sh, ref.S, impulses, 1e-3)
    st2, w, rho, eta = orc.weights(S_sh.astype(np.float64), prob.lam)
    delta = np.tensordot(w, deltas(prob, eps, U0), axes=(0, 0))
    Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
    e_iso = float(np.abs(U_a - (U0.astype(np.float64) + Mx @ delta)).max())
    assert e_iso <= U_ATOL, f"stage-isolated |dU| {e_iso:.3e}"
    assert abs(rho_a - rho) <= 1e-6 * max(abs(rho), 1.0)
    np.testing.assert_allclose(D_a, delta, rtol=0, atol=1e-6)
    pc.end_to_end(orc, prob, S_sh, S_match, eps, U0, U_a, e_iso, "IT-shard", shards=len(sizes), it=it, **info)


def test_eight_shards_of_the_paper_shaped_iteration(env, orc):
    """K = 1920 as 8 shards of 240 (one GPU's share at 8 GPUs), T = 100, SGF window 9."""
    M, torch = env
    prob = synth.c2_problem(seed=0)
    _check(M, torch, orc, prob, synth.ellipse_map(), synth.mlp_params(32, 0), synth.C2_X0,
           synth.random_controls(prob.T, 7, scale=0.2), 3, [240] * 8, impulses=True)


def test_uneven_shards_and_seeds(env, orc):
    """Shards of different sizes (and so different block counts and merge groups)."""
    M, torch = env
    prob = synth.c2_problem(seed=1)
    _check(M, torch, orc, prob, synth.ellipse_map(), synth.mlp_params(32, 0), synth.C2_X0,
           np.zeros((prob.T, 2), np.float32), 0, [700, 700, 520], impulses=True)


def test_shards_with_exploration_samples(env, orc):
    """The exploration split follows the global index: with alpha = 0.01 of K = 1920 the
    samples 1901.. are drawn around zero, i.e. the second shard's local samples 901..919."""
    M, torch = env
    prob = synth.explore_problem(seed=2)
    _check(M, torch, orc, prob, synth.ellipse_map(), synth.mlp_params(32, 0), synth.C2_X0,
           synth.random_controls(prob.T, 3, scale=0.1), 1, [1000, 920], impulses=True)


def test_plain_workload_shards_and_single_sample_shards(env, orc):
    """The plain workload (K = 256, T = 30) in shards down to a single sample."""
    M, torch = env
    prob = synth.c1_problem(seed=4)
    _check(M, torch, orc, prob, synth.ring_map(), synth.mlp_params(32, 0), synth.C1_X0,
           np.zeros((prob.T, 2), np.float32), 0, [1, 127, 64, 63, 1], impulses=False)


def test_partial_rejects_bad_arguments(env):
    M, torch = env
    prob = synth.c1_problem()
    with M.Controller(prob, synth.ring_map(), synth.mlp_params(32, 0)) as c:
        with pytest.raises(M.MppiError):
            M.mppi_iterate_partial(c.ctx, synth.C1_X0, 0)
        with pytest.raises(M.MppiError):
            M.mppi_merge_update(c.ctx, 0, 1)
        rows = torch.zeros((1, 2 + 2 * prob.T), device="cuda")
        with pytest.raises(M.MppiError):
            M.mppi_merge_update(c.ctx, rows.data_ptr(), 0)
