"""Pins of Algorithm 3 (cross-entropy weights) in the oracle: zeta = round(K (1 - delta)),
the zeta lowest-cost samples weigh 1/zeta each (ties to the lower index, non-finite
costs never elite), and the MPC iteration of Algorithm 1 with these weights."""
import itertools
import math

import numpy as np
import pytest

import synth

INF = float("inf")


def _support(w):
    return set(np.nonzero(w)[0].tolist())


@pytest.mark.parametrize("K,delta,zeta", [(1920, 0.8, 384), (10, 0.75, 3), (10, 0.85, 1), (5, 0.0, 5),
                                          (7, 0.5, 4), (100, 0.999, 0), (1, 0.4, 1)])
def test_zeta_rounds_half_away_from_zero(orc, K, delta, zeta):
    # round(K (1 - delta)) with the FP32 delta: K (1 - delta) = 2.5 exactly at K = 10,
    # delta = 0.75 (rounds up); fl32(0.85) = 0.85000002 gives 1.4999998 (rounds down)
    assert orc.cem_zeta(K, delta) == zeta


def test_worked_small_cases(orc):
    st, w, z, n = orc.weights_cem([3.0, 1.0, 2.0, 5.0, 4.0], 2)
    assert st == orc.OK and n == 2 and z == 2.0
    np.testing.assert_array_equal(w, [0, 0.5, 0.5, 0, 0])
    # ties at the threshold go to the lower sample index
    st, w, z, n = orc.weights_cem([2.0, 1.0, 2.0, 2.0, 5.0], 3)
    np.testing.assert_array_equal(w, [1 / 3, 1 / 3, 1 / 3, 0, 0])
    # non-finite costs are never elite; fewer finite costs than zeta: average over them
    st, w, z, n = orc.weights_cem([INF, 1.0, float("nan"), 2.0], 3)
    assert st == orc.OK and n == 2 and z == 2.0
    np.testing.assert_array_equal(w, [0, 0.5, 0, 0.5])
    st, w, z, n = orc.weights_cem([INF, INF], 1)
    assert st == orc.E_NONFINITE and n == 0 and not w.any()


def test_brute_force_over_orders(orc):
    # every ordering of a small cost vector with repeats: the elite set is the first zeta
    # entries of the (cost, index) order
    base = [4.0, 1.0, 3.0, 1.0, 2.0, 3.0]
    for perm in itertools.permutations(range(6)):
        S = [base[i] for i in perm]
        for zeta in range(1, 7):
            _, w, z, n = orc.weights_cem(S, zeta)
            ranked = sorted(range(6), key=lambda k: (S[k], k))
            assert _support(w) == set(ranked[:zeta])
            assert z == S[ranked[zeta - 1]] and n == zeta
            assert math.isclose(w.sum(), 1.0, rel_tol=0, abs_tol=1e-15)


def test_literal_strict_comparison_keeps_one_sample_fewer(orc):
    # Algorithm 3 compares S_k < S_zeta; with distinct costs that set is the elite set
    # minus the sample ranked zeta (the reading adds it back so the weights sum to 1)
    rng = np.random.default_rng(0)
    S = rng.normal(size=200)
    for zeta in (1, 7, 40, 200):
        _, w, z, n = orc.weights_cem(S, zeta)
        Z = np.sort(S)[zeta - 1]
        literal = set(np.nonzero(S < Z)[0].tolist())
        assert len(literal) == zeta - 1
        assert _support(w) == literal | {int(np.nonzero(S == Z)[0][0])}


def test_invariants_and_limits(orc):
    rng = np.random.default_rng(1)
    S = rng.normal(size=1000) * 50.0
    _, w, z, n = orc.weights_cem(S, 200)
    elite = w > 0
    assert elite.sum() == 200 and np.all(w[elite] == 1 / 200)
    assert S[elite].max() <= S[~elite].min() and z == S[elite].max()
    # permuting the samples permutes the weights (distinct costs)
    p = rng.permutation(1000)
    _, wp, _, _ = orc.weights_cem(S[p], 200)
    np.testing.assert_array_equal(wp, w[p])
    # zeta = K: every finite sample, uniform
    _, wK, _, _ = orc.weights_cem(S, 1000)
    np.testing.assert_array_equal(wK, np.full(1000, 1e-3))
    # zeta = 1 selects the minimum, as Algorithm 2 does for lambda -> 0
    _, w1, _, _ = orc.weights_cem(S, 1)
    _, wit, _, _ = orc.weights(S, 1e-9)
    np.testing.assert_array_equal(w1, wit)


def _small(orc, **kw):
    p = synth.with_(synth.c1_problem(), K=120, T=20, weighting=1, **kw)
    return orc.OracleProblem(p, synth.ring_map(), synth.mlp_params(32, 0)), p


def test_iteration_averages_the_elite_controls(orc):
    # U <- U + SGF * (1/zeta) sum_{k in E} delta_k: with smoothing off the new controls are
    # the plain average of the elite samples' controls u + eps (Section V)
    U = synth.random_controls(20, 1, scale=0.4)
    op, p = _small(orc, elite=0.8)
    r = orc.iterate(op, synth.C1_X0, U)
    eps = orc.noise(op, 0).astype(np.float64)
    zeta = 24                                    # round(120 * 0.2)
    elite = np.argsort(r.S, kind="stable")[:zeta]
    v = U.astype(np.float64)[None] + eps[elite]
    np.testing.assert_allclose(r.U, v.mean(axis=0), rtol=0, atol=1e-12)
    assert r.rho == np.sort(r.S)[zeta - 1] and r.eta == zeta


def test_iteration_with_smoothing_and_exploration(orc):
    U = synth.random_controls(20, 2, scale=0.4)
    op, p = _small(orc, elite=0.5, explore=0.25, sg_window=9, sg_order=2)
    r = orc.iterate(op, synth.C1_X0, U)
    eps = orc.noise(op, 0).astype(np.float64)
    d = eps.copy()
    d[90:] -= U.astype(np.float64)[None]         # samples 90..119 drawn around zero
    elite = np.argsort(r.S, kind="stable")[:60]
    M = orc.sgf_matrix(20, 9, 2)
    np.testing.assert_allclose(r.U, U + M @ d[elite].mean(axis=0), rtol=0, atol=1e-12)


@pytest.mark.parametrize("elite", [-0.1, 1.0, float("nan"), 0.999])
def test_invalid_elite_rejected(orc, elite):
    op, _ = _small(orc, elite=elite)           # 0.999: round(120 * 0.001) = 0 samples
    with pytest.raises(ValueError):
        orc.iterate(op, synth.C1_X0, np.zeros((20, 2), np.float32))


def test_objective_needs_information_theoretic_weights(orc):
    op, _ = _small(orc)
    with pytest.raises(ValueError):
        orc.objective(op, synth.C1_X0, np.zeros((20, 2)))
