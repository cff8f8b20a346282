"""Pins of Algorithm 2 (Information Theoretic Weight Computation) and the shift of
Section III-D-1: invariants, limits, and brute force in 50-digit decimal arithmetic
of the unshifted definition w = exp(-S/lambda) / sum exp(-S/lambda) (Eq. IT-Controls)."""
from decimal import Decimal, getcontext

import numpy as np
import pytest


def test_invariants(orc):
    rng = np.random.default_rng(0)
    for K in (1, 2, 7, 256, 1920):
        S = rng.uniform(10.0, 5000.0, K)
        for lam in (0.5, 6.7, 100.0):
            st, w, rho, eta = orc.weights(S, lam)
            assert st == orc.OK
            assert np.all(w >= 0)
            assert abs(w.sum() - 1.0) <= K * 2.3e-16 + 1e-15
            assert 1.0 <= eta <= K
            k = int(np.argmin(S))
            assert rho == S[k]
            assert w[k] == pytest.approx(1.0 / eta, rel=1e-15)
            # adding a constant to every cost leaves the weights unchanged
            st2, w2, _, _ = orc.weights(S + 12345.678, lam)
            np.testing.assert_allclose(w2, w, rtol=1e-9, atol=1e-300)


def test_limits(orc):
    rng = np.random.default_rng(1)
    S = rng.uniform(0.0, 10.0, 50)
    _, w, _, _ = orc.weights(S, 1e-6)                 # lambda -> 0: argmin only
    assert w[np.argmin(S)] == 1.0 and np.count_nonzero(w) == 1
    _, w, _, _ = orc.weights(S, 1e12)                 # lambda -> inf: uniform
    np.testing.assert_allclose(w, 1.0 / 50, rtol=1e-10)
    _, w, rho, eta = orc.weights(np.array([42.0]), 3.0)   # K = 1
    assert w[0] == 1.0 and eta == 1.0 and rho == 42.0


def test_brute_force_decimal(orc):
    getcontext().prec = 50
    rng = np.random.default_rng(2)
    for K in (1, 2, 3, 4):
        for lam in (0.3, 1.0, 6.7):
            S = rng.uniform(0.0, 8.0, K)
            _, w, _, _ = orc.weights(S, lam)
            e = [(-Decimal(float(s)) / Decimal(lam)).exp() for s in S]
            tot = sum(e)
            for k in range(K):
                assert abs(Decimal(float(w[k])) - e[k] / tot) < Decimal("1e-15")


def test_nonfinite_costs(orc):
    S = np.array([3.0, np.inf, 1.0, np.nan, 2.0])
    st, w, rho, eta = orc.weights(S, 1.0)
    assert st == orc.OK and w[1] == 0 and w[3] == 0 and rho == 1.0
    assert abs(w.sum() - 1.0) < 1e-15
    st, w, _, _ = orc.weights(np.array([np.inf, np.nan]), 1.0)
    assert st == orc.E_NONFINITE and np.all(w == 0)
