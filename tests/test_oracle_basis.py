"""Pins of the basis-function dynamics model (appendix; Section VI-B-1) in the oracle:
f(x_d, v) = Theta^T phi(x_d, v) with the 25 basis functions.  The basis functions are
checked through relations between them that fix every normaliser, the tan(arctan z) = z
identity of the tyre terms, the low-speed branches against library routines, the
[basis][output] layout of Theta through the plant step, and closed-form trajectories."""
import math

import numpy as np
import pytest

import synth


def _points(n=50, seed=0, vmin=0.2):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        xd = np.array([rng.normal(0, 0.2), rng.uniform(vmin, 12.0), rng.normal(0, 1.0), rng.normal(0, 1.0)])
        u = rng.uniform(-1, 1, size=2)
        yield xd, u


def test_relations_fix_every_normaliser(orc):
    for xd, u in _points():
        p = np.concatenate([[np.nan], orc.basis_phi(xd, u)])   # 1-based like the paper
        rel = lambda a, b: np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-300)
        rel(p[12], p[11] * abs(p[11]))
        rel(p[13], p[11] ** 3)
        rel(p[15], p[14] * abs(p[14]))
        rel(p[16], p[14] ** 3)
        rel(p[24], p[1] ** 2)
        rel(p[25], p[1] ** 3)
        rel(p[22], p[2] ** 2)
        rel(p[23], p[2] ** 3)
        k = 1400.0 / 1200.0
        rel(p[3], p[9] * p[11] * k)
        rel(p[4], p[3] * abs(p[11]) * k)
        rel(p[5], p[3] * (p[11] * k) ** 2)
        rel(p[6], p[7] * p[8] * 4.0)            # (r/10)(v_y/10) 100/25
        rel(p[17], p[7] * p[2] * 2.0)           # (r/10)(v_x/10) 100/50
        rel(p[19], p[18] * p[7] * 10.0)
        rel(p[20], p[18] * p[2] * 10.0 / 3.0)
        rel(p[21], p[18] * p[2] * p[7] * 20.0)  # 100 / 5
        rel(p[10], p[8] / p[2] / 40.0)
        # the raw quantities behind the normalisers
        rel(p[1], u[1])
        rel(p[2] * 10.0, xd[1])
        rel(p[7] * 10.0, xd[3])
        rel(p[8] * 10.0, xd[2])
        rel(p[18], xd[0])
        rel(p[9], math.sin(u[0]))


def test_tyre_terms_are_the_slip_tangents(orc):
    # tan(arctan z) = z: the front term is v_y/v_x + 0.45 r/v_x - u_delta, the rear
    # v_y/v_x - 0.35 r/v_x (r = heading rate)
    for xd, u in _points(seed=1):
        p = orc.basis_phi(xd, u)
        vx, vy, r = xd[1], xd[2], xd[3]
        np.testing.assert_allclose(p[10] * 1400.0, vy / vx + 0.45 * r / vx - u[0], rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(p[13] * 40.0, vy / vx - 0.35 * r / vx, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("vx", [0.1, 0.05, 0.0, -2.0])
def test_low_speed_branches(orc, vx):
    # v_x <= 0.1 (strictly not above): alpha_f = -u_delta, alpha_r = 0, phi_10 = 0
    xd = np.array([0.1, vx, 0.7, -0.4])
    u = np.array([0.3, -0.6])
    p = orc.basis_phi(xd, u)
    np.testing.assert_allclose(p[10] * 1400.0, -math.tan(0.3), rtol=1e-15)
    assert p[9] == 0.0 and p[13] == 0.0 and p[14] == 0.0 and p[15] == 0.0
    # just above the threshold the moving branch applies
    p2 = orc.basis_phi(np.array([0.1, 0.1000001, 0.7, -0.4]), u)
    assert p2[9] != 0.0 and p2[13] != 0.0


def _basis_op(orc, theta, **kw):
    kw = {"K": 4, "T": 20, "model": 1, **kw}
    prob = synth.with_(synth.c1_problem(), **kw)
    return orc.OracleProblem(prob, synth.ring_map(), theta), prob


def test_theta_layout_through_the_plant_step(orc):
    # Theta = e_{i,o}: one Euler step changes only dynamic state o, by dt * phi_i
    x = np.array([0.0, 0.0, 0.3, 0.05, 5.0, 0.4, -0.2])
    u = np.array([0.2, 0.5])
    phi = orc.basis_phi(x[3:], u)
    for i in (0, 4, 10, 13, 20, 24):
        for o in range(4):
            th = np.zeros((25, 4), np.float32)
            th[i, o] = 1.0
            op, prob = _basis_op(orc, th)
            xn = orc.plant_step(op, x, u)
            dd = xn[3:] - x[3:]
            exp = np.zeros(4)
            exp[o] = np.float32(prob.dt) * phi[i]
            np.testing.assert_allclose(dd, exp, rtol=1e-9, atol=1e-15)


def test_linear_in_theta(orc):
    x = np.array([1.0, 2.0, 0.3, 0.05, 5.0, 0.4, -0.2])
    u = np.array([-0.3, 0.4])
    full = synth.basis_theta(1)
    t1, t2 = full.copy(), full.copy()      # disjoint supports: the FP32 sum is exact
    t1[13:] = 0.0
    t2[:13] = 0.0
    d = [orc.plant_step(_basis_op(orc, t)[0], x, u)[3:] - x[3:] for t in (t1, t2, t1 + t2)]
    np.testing.assert_allclose(d[2], d[0] + d[1], rtol=1e-9, atol=1e-12)


def test_closed_form_trajectories(orc):
    T = 20
    # throttle only: v_x ramps linearly, v_x(t) = v_x0 + c u_F dt t
    th = np.zeros((25, 4), np.float32)
    th[0, 1] = 2.0
    op, prob = _basis_op(orc, th, T=T)
    U = np.tile(np.array([[0.0, 0.5]], np.float32), (T, 1))
    x0 = np.array([0, 0, 0, 0, 3.0, 0, 0], np.float32)
    _, tr = orc.rollout(op, x0, U, np.zeros((4, T, 2), np.float32), traj=True)
    dt = float(np.float32(prob.dt))
    np.testing.assert_allclose(tr[0, :, 4], 3.0 + 2.0 * 0.5 * dt * np.arange(T + 1), rtol=1e-12)
    # drag only: v_x decays geometrically, v_x(t) = v_x0 (1 - k dt)^t with phi_2 = v_x/10
    th = np.zeros((25, 4), np.float32)
    th[1, 1] = -5.0                                   # dv_x/dt = -0.5 v_x
    op, _ = _basis_op(orc, th, T=T)
    _, tr = orc.rollout(op, x0, U, np.zeros((4, T, 2), np.float32), traj=True)
    np.testing.assert_allclose(tr[0, :, 4], 3.0 * (1.0 - 0.5 * dt) ** np.arange(T + 1), rtol=1e-12)
    # the heading follows the heading rate, the position the body-frame velocity
    assert np.all(tr[0, :, 2] == 0.0) and np.allclose(tr[0, :, 1], 0.0)


def test_basis_model_rejections(orc):
    op, _ = _basis_op(orc, synth.basis_theta(0), model=2)
    with pytest.raises(ValueError):
        orc.iterate(op, synth.C1_X0, np.zeros((20, 2), np.float32))
    op, _ = _basis_op(orc, synth.basis_theta(0))
    with pytest.raises(ValueError):
        orc.objective(op, synth.C1_X0, np.zeros((20, 2)))
