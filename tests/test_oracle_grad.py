"""Pins of the oracle's gradient of the free-energy objective
J = -lambda log((1/K) sum_k exp(-S_k/lambda))  (Eq. FreeEnergy, Monte-Carlo estimate)
with respect to the nominal controls and the network parameters: central finite
differences of the oracle's own FP64 objective (which never uses the adjoint), the
K = 1 case (J = S_1) and the relation dJ/dS_k = w_k."""
import numpy as np
import pytest

import synth


def _setup(orc, K=48, T=16, seed=0, lam=1.0):
    p = synth.with_(synth.c5_problem(seed=seed), K=K, T=T, lam=lam)
    params = synth.mlp_params(32, seed=seed)
    op = orc.OracleProblem(p, synth.ring_map(), params)
    U = synth.random_controls(T, seed, scale=0.2).astype(np.float64)
    return op, p, params, U


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(orc, seed):
    op, p, params, U = _setup(orc, seed=seed)
    x0 = synth.C1_X0
    J, gU, gth = orc.objective_grad(op, x0, U)
    J2, _ = orc.objective(op, x0, U)
    assert J == pytest.approx(J2, rel=1e-14)
    rng = np.random.default_rng(100 + seed)
    h = 1e-6
    eps = orc.noise(op, 0)
    V = U[None] + eps
    checked = 0
    for idx in rng.choice(U.size, 12, replace=False):
        t, c = divmod(int(idx), 2)
        # skip coordinates where some sample sits within h of a clamp kink
        if np.any(np.abs(np.abs(V[:, t, c]) - 1.0) < 10 * h):
            continue
        d = np.zeros_like(U)
        d[t, c] = h
        fd = (orc.objective(op, x0, U + d)[0] - orc.objective(op, x0, U - d)[0]) / (2 * h)
        assert gU[t, c] == pytest.approx(fd, rel=2e-5, abs=2e-6), (t, c)
        checked += 1
    assert checked >= 6
    P = params.astype(np.float64)
    for idx in rng.choice(P.size, 12, replace=False):
        d = np.zeros_like(P)
        d[idx] = h
        fd = (orc.objective(op, x0, U, params=P + d)[0] - orc.objective(op, x0, U, params=P - d)[0]) / (2 * h)
        assert gth[idx] == pytest.approx(fd, rel=2e-5, abs=2e-6), idx


def test_single_sample_gradient_is_cost_gradient(orc):
    op, p, params, U = _setup(orc, K=1, T=10)
    J, gU, _ = orc.objective_grad(op, synth.C1_X0, U)
    _, S = orc.objective(op, synth.C1_X0, U)
    assert J == pytest.approx(S[0], rel=1e-13)
    h = 1e-6
    d = np.zeros_like(U)
    d[3, 1] = h
    fd = (orc.objective(op, synth.C1_X0, U + d)[1][0] - orc.objective(op, synth.C1_X0, U - d)[1][0]) / (2 * h)
    assert gU[3, 1] == pytest.approx(fd, rel=1e-5, abs=1e-7)


def test_objective_is_softmin_of_costs(orc):
    op, p, params, U = _setup(orc, K=32, T=12, lam=2.5)
    J, S = orc.objective(op, synth.C1_X0, U)
    ref = -2.5 * np.log(np.mean(np.exp(-(S - S.min()) / 2.5))) + S.min()
    assert J == pytest.approx(ref, rel=1e-13)
    assert S.min() - 1e-12 <= J <= S.mean() + 1e-9        # softmin lies between min and mean


@pytest.mark.slow
@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_gradient_full_shape_central_differences(orc, seed):
    """The differentiation workload's own shape (K=4096, T=100, h=32, the smooth ring-map
    cost): the oracle's reverse-mode gradient against FP64 central differences with
    h = 1e-6 on 32 random coordinates (16 of U, 16 of the network parameters), each within
    2e-5 relative + 2e-6 absolute.  A coordinate outside that bar is reported instead of
    failed only if the difference step straddles a kink (a clamp, or a bilinear cell edge
    of the map): its second difference at h is then far above the one that the curvature
    measured at 10 h predicts.  At most 2 such coordinates are allowed."""
    import os
    p = synth.c5_problem(seed=seed)
    params = synth.mlp_params(32, seed=seed)
    op = orc.OracleProblem(p, synth.ring_map(), params, nthreads=os.cpu_count() or 1)
    U = synth.random_controls(p.T, seed, scale=0.2).astype(np.float64)
    x0 = synth.C1_X0
    J0, gU, gth = orc.objective_grad(op, x0, U)
    rng = np.random.default_rng(1000 + seed)
    h = 1e-6
    P = params.astype(np.float64)
    coords = [("U", int(i)) for i in rng.choice(U.size, 16, replace=False)] + \
             [("theta", int(i)) for i in rng.choice(P.size, 16, replace=False)]

    def J_at(kind, idx, step):
        if kind == "U":
            d = np.zeros_like(U)
            d.flat[idx] = step
            return orc.objective(op, x0, U + d)[0]
        d = np.zeros_like(P)
        d[idx] = step
        return orc.objective(op, x0, U, params=P + d)[0]

    kinks = []
    for kind, idx in coords:
        Jp, Jm = J_at(kind, idx, h), J_at(kind, idx, -h)
        g = gU.flat[idx] if kind == "U" else gth[idx]
        fd = (Jp - Jm) / (2 * h)
        if abs(g - fd) <= 2e-5 * abs(fd) + 2e-6:
            continue
        second_h = abs(Jp - 2 * J0 + Jm) / h
        second_10h = abs(J_at(kind, idx, 10 * h) - 2 * J0 + J_at(kind, idx, -10 * h)) / (10 * h)
        straddles = second_h > 10 * (second_10h / 10) + 1e-6   # ten times the smooth prediction
        print(f"seed {seed}: {kind}[{idx}] fd {fd:.6e} adjoint {g:.6e}; second differences /step at h "
              f"{second_h:.3e}, at 10h {second_10h:.3e}; kink: {straddles}", flush=True)
        assert straddles, (kind, idx, fd, g)
        kinks.append((kind, idx))
    assert len(kinks) <= 2
