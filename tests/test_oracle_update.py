"""Pins of the control update of Algorithm 1 (U <- U + SGF * sum_k w_k E^k), the
Savitzky-Golay filter (Section III-D-4), the warm-start shift, and the information-
theoretic control law itself on a linear-Gaussian/quadratic toy whose optimum is known
in closed form (Eqs. Optimal-Density, QuadraticOptimization, IT-Controls)."""
import math
from fractions import Fraction
from pathlib import Path

import numpy as np
import pytest
from scipy.signal import savgol_filter

import synth

GOLD = Path(__file__).resolve().parent / "golden"


def _golden(name):
    out = {}
    for line in (GOLD / name).read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            key, *vals = line.split()
            out[key] = vals
    return out


def test_sg_centre_taps_match_published_table(orc):
    g = _golden("sg_taps_w9_o2.txt")
    taps = np.array([int(v) for v in g["taps"]], dtype=np.float64) / int(g["norm"][0])
    M = orc.sgf_matrix(30, 9, 2)
    for t in range(4, 26):
        np.testing.assert_allclose(M[t, t - 4:t + 5], taps, rtol=0, atol=1e-14)
    # order 3 has the same centre taps
    M3 = orc.sgf_matrix(30, 9, 3)
    np.testing.assert_allclose(M3[15, 11:20], taps, atol=1e-13)


@pytest.mark.parametrize("T,window,order", [(9, 9, 2), (30, 9, 2), (100, 9, 2), (50, 5, 3), (20, 7, 1)])
def test_sg_matches_scipy_interp_mode(orc, T, window, order):
    M = orc.sgf_matrix(T, window, order)
    rng = np.random.default_rng(T + window)
    for _ in range(5):
        x = rng.normal(size=T)
        ref = savgol_filter(x, window, order, mode="interp")
        np.testing.assert_allclose(M @ x, ref, rtol=0, atol=1e-12)


def test_sg_reproduces_polynomials_and_window1_identity(orc):
    T = 40
    M = orc.sgf_matrix(T, 9, 2)
    t = np.arange(T, dtype=np.float64)
    for poly in (np.ones(T), t, 0.5 * t ** 2 - 3 * t + 2):
        np.testing.assert_allclose(M @ poly, poly, atol=1e-9)
    np.testing.assert_array_equal(orc.sgf_matrix(T, 1, 0), np.eye(T))


def test_shift(orc):
    U = np.arange(10, dtype=np.float64).reshape(5, 2)
    Uo, u0 = orc.shift(U)
    np.testing.assert_array_equal(u0, [0, 1])
    np.testing.assert_array_equal(Uo[:4], U[1:])
    np.testing.assert_array_equal(Uo[4], [0, 0])


def _small(orc, **kw):
    p = synth.with_(synth.c1_problem(), K=64, T=20, **kw)
    return orc.OracleProblem(p, synth.ring_map(), synth.mlp_params(32, 0)), p


def test_sigma_to_zero_leaves_controls_unchanged(orc):
    U = synth.random_controls(20, 3)
    prev = None
    for s in (1e-2, 1e-4, 1e-6):
        op, p = _small(orc, sigma2=(0.3 * s, 0.35 * s), sg_window=9, sg_order=2)
        r = orc.iterate(op, synth.C1_X0, U)
        eps = orc.noise(op, 0)
        dU = np.abs(r.U - U.astype(np.float64)).max()
        bound = np.abs(orc.sgf_matrix(20, 9, 2)).sum(axis=1).max() * np.abs(eps).max()
        assert dU <= bound * (1 + 1e-12)
        if prev is not None:
            assert dU < prev * 0.2          # shrinks like sqrt(s)
        prev = dU


def test_lambda_to_zero_selects_argmin(orc):
    op, p = _small(orc, lam=1e-7, sg_window=9, sg_order=2)
    U = synth.random_controls(20, 4)
    r = orc.iterate(op, synth.C1_X0, U)
    eps = orc.noise(op, 0).astype(np.float64)
    k = int(np.argmin(r.S))
    M = orc.sgf_matrix(20, 9, 2)
    np.testing.assert_allclose(r.U, U + M @ eps[k], rtol=0, atol=1e-12)


def test_update_is_weighted_average_of_noise(orc):
    op, p = _small(orc, lam=3.0)
    U = synth.random_controls(20, 5)
    r = orc.iterate(op, synth.C1_X0, U)
    eps = orc.noise(op, 0).astype(np.float64)
    np.testing.assert_allclose(r.delta, np.tensordot(r.w, eps, axes=(0, 0)), atol=1e-15)
    np.testing.assert_allclose(r.U, U + r.delta, atol=1e-15)
    st, w, rho, eta = orc.weights(r.S, 3.0)
    np.testing.assert_array_equal(w, r.w)


def test_nonfinite_iteration_leaves_controls(orc):
    p = synth.with_(synth.c1_problem(), K=16, T=10)
    nan_map = synth.constant_map(float("nan"))
    op = orc.OracleProblem(p, nan_map, synth.mlp_params(32, 0))
    U = synth.random_controls(10, 6)
    r = orc.iterate(op, synth.C1_X0, U)
    assert r.status == orc.E_NONFINITE
    np.testing.assert_array_equal(r.U, U.astype(np.float64))
    assert np.all(np.isinf(r.S))


def _lqg_closed_form(a, b, q, lam, sig2, x0, T):
    G = np.zeros((T, T))
    for t in range(T):
        for s in range(t + 1):
            G[t, s] = a ** (t - s) * b
    h = np.array([a ** (t + 1) * x0 for t in range(T)])
    Q = q * np.eye(T)
    return -np.linalg.solve(G.T @ Q @ G + 0.5 * lam / sig2 * np.eye(T), G.T @ Q @ h)


def test_lqg_closed_form_values_match_golden():
    g = _golden("lqg_toy.txt")
    np.testing.assert_allclose(_lqg_closed_form(1, 1, 1, 1, 1, 1, 1), [float(Fraction(v)) for v in g["T1"]], rtol=1e-14)
    np.testing.assert_allclose(_lqg_closed_form(1, 1, 1, 1, 1, 1, 2), [float(Fraction(v)) for v in g["T2"]], rtol=1e-14)


@pytest.mark.parametrize("U0", [-2.0 / 3.0, 0.5, -2.0])
def test_lqg_toy_one_iteration_reaches_optimum(orc, U0):
    """One importance-sampled iteration from any U0 estimates E_{Q*}[v] = U*; the
    control-cost term gamma u^T Sigma^-1 eps (gamma = lambda) is what removes the
    dependence on the sampling mean."""
    K = 1 << 21
    Ustar = float(Fraction(_golden("lqg_toy.txt")["T1"][0]))
    Uo = orc.toy_iterate(1.0, 1.0, 1.0, 1.0, 1.0, 1.0, np.array([U0]), K, seed=3)
    assert abs(Uo[0] - Ustar) < 5e-3, Uo


def test_lqg_toy_two_steps_and_general(orc):
    K = 1 << 21
    g = _golden("lqg_toy.txt")
    Ustar = [float(Fraction(v)) for v in g["T2"]]
    Uo = orc.toy_iterate(1.0, 1.0, 1.0, 1.0, 1.0, 1.0, np.array([0.3, -0.4]), K, seed=4)
    np.testing.assert_allclose(Uo, Ustar, atol=6e-3)
    a, b, q, lam, s2, x0 = 0.9, 0.5, 2.0, 1.5, float(np.float32(0.7)), 1.2
    ref = _lqg_closed_form(a, b, q, lam, s2, x0, 3)
    Uo = orc.toy_iterate(a, b, q, lam, s2, x0, np.array([0.1, 0.0, -0.2]), K, seed=5)
    np.testing.assert_allclose(Uo, ref, atol=6e-3)


def test_lqg_toy_catches_missing_control_cost(orc):
    """Planted mistake (in the oracle, on the CPU): without the control-cost term the
    estimate is the mean of exp(-S/lambda) N(U0, Sigma), which at T = 1 and
    a = b = q = lambda = Sigma = x0 = 1 is (U0 - 2)/3, not U* = -2/3."""
    K = 1 << 20
    good = orc.toy_iterate(1.0, 1.0, 1.0, 1.0, 1.0, 1.0, np.array([-2.0]), K, seed=6)[0]
    bad = orc.toy_iterate(1.0, 1.0, 1.0, 1.0, 1.0, 1.0, np.array([-2.0]), K, seed=6, ctrl_scale=0.0)[0]
    assert abs(good + 2.0 / 3.0) < 5e-3
    assert abs(bad - (-4.0 / 3.0)) < 5e-3
    bad_sign = orc.toy_iterate(1.0, 1.0, 1.0, 1.0, 1.0, 1.0, np.array([-2.0]), K, seed=6, ctrl_scale=-1.0)[0]
    assert abs(bad_sign + 2.0 / 3.0) > 0.3
