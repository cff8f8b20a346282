"""Pins of the exploration samples of Algorithm 1 (zero-mean samples for k >= (1-alpha)K,
Section IV's disturbance discussion) and of the decoupled control-cost weight gamma
(Section III-D-2) in the oracle.

The oracle writes the per-step control cost as gamma u^T Sigma^-1 (v - u) and the update
as U + SGF * sum_k w_k (v_k - u); the tests check these against the paper's own forms:
the v form of the running cost (Algorithm 1), which may differ only by a constant shared
by all samples, and the optimal-control law u* = sum_k w_k v_k of Eq. IT-Controls."""
import numpy as np
import pytest

import synth


def _op(orc, **kw):
    p = synth.with_(synth.c1_problem(), K=100, T=20, **kw)
    return orc.OracleProblem(p, synth.ring_map(), synth.mlp_params(32, 0)), p


def _v_controls(U, eps, n_imp):
    """v_{k,t}: u_t + eps for the first n_imp samples, eps alone for the rest."""
    v = eps.astype(np.float64).copy()
    v[:n_imp] += U.astype(np.float64)[None]
    return v


def test_exploration_samples_are_the_last_ones(orc):
    # alpha = 1/4 and K = 100: (1 - alpha) K = 75 exactly, so samples 75..99 are drawn
    # around zero.  With gamma = 0 the cost of a sample depends on U only through the
    # dynamics, so an exploration sample's cost equals its cost at U = 0.
    U = synth.random_controls(20, 1, scale=0.5)
    Z = np.zeros_like(U)
    op_a, _ = _op(orc, gamma=0.0, explore=0.25)
    op_0, _ = _op(orc, gamma=0.0, explore=0.0)
    eps = orc.noise(op_0, 0)
    S_a = orc.rollout(op_a, synth.C1_X0, U, eps)
    S_u = orc.rollout(op_0, synth.C1_X0, U, eps)
    S_z = orc.rollout(op_0, synth.C1_X0, Z, eps)
    np.testing.assert_array_equal(S_a[:75], S_u[:75])
    np.testing.assert_array_equal(S_a[75:], S_z[75:])
    assert np.all(S_u[75:] != S_z[75:])      # U matters for those samples without alpha


@pytest.mark.parametrize("K,alpha,n_explore", [(64, 1 / 64, 1), (64, 0.5 / 64, 0), (1920, 0.01, 19),
                                               (100, 0.1, 10), (7, 1.0, 7), (7, 0.0, 0)])
def test_exploration_count(orc, K, alpha, n_explore):
    # The number of zero-mean samples is K - ceil((1 - alpha) K), i.e. floor(alpha K) when
    # alpha K is not an integer; found here as the samples whose cost ignores U.
    p = synth.with_(synth.c1_problem(), K=K, T=5, gamma=0.0, explore=float(np.float32(alpha)))
    op = orc.OracleProblem(p, synth.ring_map(), synth.mlp_params(32, 0))
    op0 = orc.OracleProblem(synth.with_(p, explore=0.0), synth.ring_map(), synth.mlp_params(32, 0))
    eps = orc.noise(op0, 0)
    U = synth.random_controls(5, 2, scale=0.5)
    S = orc.rollout(op, synth.C1_X0, U, eps)
    S_u = orc.rollout(op0, synth.C1_X0, U, eps)
    S_z = orc.rollout(op0, synth.C1_X0, np.zeros_like(U), eps)
    ignores_u = (S == S_z) & (S != S_u)
    follows_u = (S == S_u) & (S != S_z)
    assert np.all(ignores_u | follows_u)
    assert np.array_equal(np.nonzero(ignores_u)[0], np.arange(K - n_explore, K))


def test_running_cost_is_the_paper_v_form_up_to_a_constant(orc):
    # Algorithm 1 accumulates c(x) + gamma u^T Sigma^-1 v.  The state part is the cost with
    # gamma = 0 (gamma does not enter the dynamics); the control part is written out from v.
    U = synth.random_controls(20, 3, scale=0.4)
    gam, sig2 = 0.7, np.array([0.3, 0.35])
    # the problem holds them in FP32
    gam32, sig2_32 = float(np.float32(gam)), np.float32(sig2).astype(np.float64)
    op, p = _op(orc, gamma=gam, explore=0.25)
    op_c, _ = _op(orc, gamma=0.0, explore=0.25)
    eps = orc.noise(op, 0)
    S = orc.rollout(op, synth.C1_X0, U, eps)
    S_state = orc.rollout(op_c, synth.C1_X0, U, eps)
    v = _v_controls(U, eps, 75)
    S_paper = S_state + gam32 * np.einsum("tc,ktc->k", U.astype(np.float64) / sig2_32, v)
    offset = S - S_paper
    const = -gam32 * np.sum(U.astype(np.float64) ** 2 / sig2_32)
    np.testing.assert_allclose(offset, const, rtol=0, atol=1e-9 * np.abs(S).max())
    # hence the same weights as the paper's form
    _, w_paper, _, _ = orc.weights(S_paper, p.lam)
    r = orc.iterate(op, synth.C1_X0, U)
    np.testing.assert_allclose(r.w, w_paper, rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("alpha", [0.0, 0.25, 1.0])
def test_update_is_weighted_average_of_controls(orc, alpha):
    # Eq. IT-Controls: u*_t = sum_k w_k v_{k,t} (no smoothing), whatever mix of samples.
    U = synth.random_controls(20, 4, scale=0.4)
    op, p = _op(orc, lam=3.0, gamma=0.5, explore=alpha)
    r = orc.iterate(op, synth.C1_X0, U)
    eps = orc.noise(op, 0)
    n_imp = 100 - int(round(alpha * 100))
    v = _v_controls(U, eps, n_imp)
    np.testing.assert_allclose(r.U, np.tensordot(r.w, v, axes=(0, 0)), rtol=0, atol=1e-12)
    np.testing.assert_allclose(r.delta, r.U - U.astype(np.float64), rtol=0, atol=1e-12)


def test_all_exploration_with_gamma_zero_forgets_u(orc):
    # Every sample around zero and no control cost: the costs, the weights and the
    # optimal controls sum_k w_k eps_k do not depend on U.  With smoothing the new
    # controls are SGF * that + (I - SGF) U.
    U1 = synth.random_controls(20, 5, scale=0.4)
    U2 = synth.random_controls(20, 6, scale=0.4)
    op, _ = _op(orc, gamma=0.0, explore=1.0, sg_window=9, sg_order=2)
    r1 = orc.iterate(op, synth.C1_X0, U1)
    r2 = orc.iterate(op, synth.C1_X0, U2)
    np.testing.assert_array_equal(r1.S, r2.S)
    eps = orc.noise(op, 0).astype(np.float64)
    ustar = np.tensordot(r1.w, eps, axes=(0, 0))
    M = orc.sgf_matrix(20, 9, 2)
    for U, r in ((U1, r1), (U2, r2)):
        U = U.astype(np.float64)
        np.testing.assert_allclose(r.U, M @ ustar + (np.eye(20) - M) @ U, rtol=0, atol=1e-12)


def test_u_zero_makes_exploration_irrelevant(orc):
    op_a, _ = _op(orc, gamma=0.3, explore=0.25, sg_window=9, sg_order=2)
    op_0, _ = _op(orc, gamma=0.3, explore=0.0, sg_window=9, sg_order=2)
    Z = np.zeros((20, 2), dtype=np.float32)
    ra, r0 = orc.iterate(op_a, synth.C1_X0, Z), orc.iterate(op_0, synth.C1_X0, Z)
    np.testing.assert_array_equal(ra.S, r0.S)
    np.testing.assert_array_equal(ra.U, r0.U)


@pytest.mark.parametrize("alpha", [-0.01, 1.01, float("nan")])
def test_invalid_fraction_rejected(orc, alpha):
    op, _ = _op(orc, explore=alpha)
    with pytest.raises(ValueError):
        orc.iterate(op, synth.C1_X0, np.zeros((20, 2), dtype=np.float32))


def test_objective_needs_importance_samples_only(orc):
    op, _ = _op(orc, explore=0.25)
    with pytest.raises(ValueError):
        orc.objective(op, synth.C1_X0, np.zeros((20, 2)))
    with pytest.raises(ValueError):
        orc.objective_grad(op, synth.C1_X0, np.zeros((20, 2)))


def test_paper_parameter_problem(orc):
    # The parameter-table problem (19 of 1920 samples explore, Savitzky-Golay 9/2): the new
    # controls are U + SGF * (sum_k w_k v_k - U).
    p = synth.explore_problem(0)
    op = orc.OracleProblem(p, synth.ellipse_map(), synth.mlp_params(32, 0))
    U = synth.random_controls(100, 7, scale=0.2)
    x0 = synth.ellipse_pose(0.3, 6.0)
    r = orc.iterate(op, x0, U)
    assert r.status == orc.OK
    assert abs(r.w.sum() - 1.0) < 1e-12
    v = _v_controls(U, orc.noise(op, 0), 1901)
    M = orc.sgf_matrix(100, 9, 2)
    U64 = U.astype(np.float64)
    np.testing.assert_allclose(r.U, U64 + M @ (np.tensordot(r.w, v, axes=(0, 0)) - U64),
                               rtol=0, atol=1e-12)
