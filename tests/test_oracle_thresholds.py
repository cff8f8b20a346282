"""Pins of the oracle's threshold bookkeeping (oracle.cpp: orc_threshold_events,
orc_threshold_margins), which decides how the parity checks treat the impulse terms of
the state cost (Section VI-C): crash_cost * 0.9^t * [h > map_thresh] and
slip_cost * [|zeta| > slip_thresh] at the post-step states t = 1..T.

* A constant map at a known distance from map_thresh: every step is a near-threshold
  crash term exactly when the window exceeds that distance, the margin is that distance,
  and the term's size is crash_cost * fl32(0.9^t) with t the post-step index.
* Zero network output (constant v_x, v_y): zeta is constant and known in closed form, so
  the slip margin and the slip terms are known; |v_x| enters, not v_x.
* A linearly growing v_y placed so that the PRE-step state x_0 sits exactly on the slip
  threshold: the margin must be measured at t = 1..T (a margin taken at the pre-step
  states would be 0), and equals the closed form at t = 1.
* With an unbounded window every step of every sample is listed, and removing the taken
  terms from S gives the cost computed with the impulses switched off.
"""
import math

import numpy as np
import pytest

import synth


def _zero_output(params, hidden, b3=(0, 0, 0, 0)):
    params = params.copy()
    n_before = 6 * hidden + hidden + hidden * hidden + hidden
    params[n_before:n_before + 4 * hidden] = 0.0
    params[-4:] = np.float32(b3)
    return params


def _prob(K=4, T=20, **cost):
    base = synth.c2_cost()
    for k, v in cost.items():
        setattr(base, k, v)
    return synth.with_(synth.c2_problem(), K=K, T=T, sg_window=1, sg_order=0, cost=base)


@pytest.mark.parametrize("delta", [3e-5, -3e-5, 2e-3])
def test_constant_map_crash_terms(orc, delta):
    thr = float(np.float32(0.99))
    c = float(np.float32(thr + delta))
    dist = abs(c - thr)
    T = 20
    p = _prob(T=T, slip_thresh=float("inf"))
    op = orc.OracleProblem(p, synth.constant_map(c), synth.mlp_params(32, 0))
    x0 = np.array([10.0, 10.0, 0.3, 0.0, 4.0, 0.0, 0.0], np.float32)
    U = np.zeros((T, 2), np.float32)
    eps = orc.noise(op, 0)
    m = orc.threshold_margins(op, x0, U, eps)
    np.testing.assert_allclose(m, dist, rtol=0, atol=0)
    ev = orc.threshold_events(op, x0, U, eps, window=1e-4)
    decay = [float(np.float32(float(np.float32(0.9)) ** t)) for t in range(T + 1)]
    for k in range(p.K):
        if dist < 1e-4:
            assert ev.n[k] == T
            np.testing.assert_array_equal(ev.t[k], np.arange(1, T + 1))
            assert np.all(ev.kind[k] == 0)
            np.testing.assert_array_equal(ev.on[k], np.full(T, int(c > thr)))
            np.testing.assert_allclose(ev.value[k], [1e4 * decay[t] for t in range(1, T + 1)], rtol=1e-15)
        else:
            assert ev.n[k] == 0
    # a window just below the distance lists nothing, just above lists every step
    assert np.all(orc.threshold_events(op, x0, U, eps, window=dist * 0.999).n == 0)
    assert np.all(orc.threshold_events(op, x0, U, eps, window=dist * 1.001).n == T)


@pytest.mark.parametrize("vx,vy", [(6.0, 2.5), (-6.0, 2.5), (3.0, -4.0)])
@pytest.mark.parametrize("offset", [4e-5, -4e-5])
def test_constant_slip_angle(orc, vx, vy, offset):
    """W3 = 0, b3 = 0: x_d is constant, zeta = -atan2(v_y, |v_x|) at every step."""
    T = 15
    zeta = -math.atan2(vy, abs(vx))
    thr = float(np.float32(abs(zeta) + offset))
    dist = abs(abs(zeta) - thr)
    p = _prob(T=T, map_thresh=float("inf"), slip_thresh=thr)
    params = _zero_output(synth.mlp_params(32, 0), 32)
    op = orc.OracleProblem(p, synth.constant_map(0.1), params)
    x0 = np.array([10.0, 10.0, 0.0, 0.0, vx, vy, 0.0], np.float32)
    U = np.zeros((T, 2), np.float32)
    eps = orc.noise(op, 0)
    m = orc.threshold_margins(op, x0, U, eps)
    np.testing.assert_allclose(m, dist, rtol=1e-12)
    ev = orc.threshold_events(op, x0, U, eps, window=1e-4)
    for k in range(p.K):
        assert ev.n[k] == T
        assert np.all(ev.kind[k] == 1)
        np.testing.assert_array_equal(ev.on[k], np.full(T, int(abs(zeta) > thr)))
        np.testing.assert_allclose(ev.value[k], 1e4)


def test_margin_is_taken_after_the_step(orc):
    """v_y(t) = v_y0 + a t dt with v_x constant (zero network weights, b3 = (0, 0, a, 0)); the
    threshold is |zeta| of the pre-step state x_0, so the margin over t = 1..T is
    |zeta(1)| - |zeta(0)| (|zeta| grows with t), not 0."""
    T, dt, a = 10, 0.02, 0.5
    vx, vy0 = 5.0, 1.0
    params = _zero_output(synth.mlp_params(32, 0), 32, b3=(0.0, 0.0, a, 0.0))
    a32, dt32 = float(np.float32(a)), float(np.float32(dt))
    z0 = math.atan2(vy0, vx)
    thr = float(np.float32(z0))
    p = _prob(K=2, T=T, map_thresh=float("inf"), slip_thresh=thr, crash_cost=0.0)
    op = orc.OracleProblem(p, synth.constant_map(0.1), params)
    x0 = np.array([10.0, 10.0, 0.0, 0.0, vx, vy0, 0.0], np.float32)
    U = np.zeros((T, 2), np.float32)
    eps = orc.noise(op, 0)
    m = orc.threshold_margins(op, x0, U, eps)
    z1 = math.atan2(vy0 + a32 * dt32, vx)
    np.testing.assert_allclose(m, abs(z1 - thr), rtol=1e-9)
    assert m.min() > 1e-3
    ev = orc.threshold_events(op, x0, U, eps, window=1.5 * abs(z1 - thr))
    for k in range(2):
        assert list(ev.t[k]) == [1]           # only the first post-step state is that close
        assert ev.on[k][0] == 1


def test_unbounded_window_removes_every_impulse(orc):
    """window = inf lists every step: S minus the taken terms is the cost without impulses."""
    p = synth.with_(synth.c2_problem(seed=3), K=64, T=60)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    op = orc.OracleProblem(p, cmap, params)
    U = synth.random_controls(60, 7, scale=0.4)
    eps = orc.noise(op, 0)
    x0 = synth.C2_X0.copy()
    x0[2], x0[4] = 0.0, 8.0      # heading across the track at 8 m/s: most samples hit the wall
    S = orc.rollout(op, x0, U, eps)
    ev = orc.threshold_events(op, x0, U, eps, window=float("inf"), cap=2 * p.T)
    assert np.all(ev.n == 2 * p.T)
    assert ev.taken().max() > 0                 # some sample leaves the track or slips
    cost0 = synth.c2_cost()
    cost0.crash_cost = 0.0
    cost0.slip_cost = 0.0
    op0 = orc.OracleProblem(synth.with_(p, cost=cost0), cmap, params)
    S0 = orc.rollout(op0, x0, U, eps)
    np.testing.assert_allclose(S - ev.taken(), S0, rtol=1e-12, atol=1e-9)
    # the crash terms carry 1e4 * fl32(0.9^t) for post-step t
    decay = np.array([float(np.float32(float(np.float32(0.9)) ** t)) for t in range(p.T + 1)])
    for k in range(4):
        crash = ev.kind[k] == 0
        np.testing.assert_allclose(ev.value[k][crash], 1e4 * decay[ev.t[k][crash]], rtol=1e-15)


def test_cap_overflow_is_reported(orc):
    thr = float(np.float32(0.99))
    p = _prob(T=20, slip_thresh=float("inf"))
    op = orc.OracleProblem(p, synth.constant_map(thr), synth.mlp_params(32, 0))
    x0 = np.array([10.0, 10.0, 0.3, 0.0, 4.0, 0.0, 0.0], np.float32)
    eps = orc.noise(op, 0)
    with pytest.raises(ValueError):
        orc.threshold_events(op, x0, np.zeros((20, 2), np.float32), eps, window=1e-4, cap=5)


def test_checker_on_the_fp32_oracle(orc):
    """The parity checker's cost bar, exercised on the CPU with the oracle's FP32
    instantiation standing in for an FP32 computation: its costs match the FP64 oracle
    once near-threshold terms may take either side, and a planted mistake -- one impulse
    term added to a sample that is far from every threshold, or a near-threshold term
    counted twice -- is caught."""
    import parity_checks as pc
    p = synth.with_(synth.c2_problem(seed=1), K=1024, T=100)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    op = orc.OracleProblem(p, cmap, params)
    U = synth.random_controls(100, 11, scale=0.35)
    eps = orc.noise(op, 0)
    x0 = synth.C2_X0.copy()
    x0[2], x0[4] = 0.8, 6.0      # heading across the track: many samples graze the crash threshold
    S64 = orc.rollout(op, x0, U, eps)
    S32 = orc.rollout(op, x0, U, eps, precision="f32")
    S_match, err, info = pc.check_costs(orc, op, p, cmap, params, x0, U, eps, S32, S64, True, 0.0)
    print(info, float(err.max()))
    assert info["n_near_threshold"] > 0
    ev = orc.threshold_events(op, x0, U, eps, window=pc.NEAR_WINDOW, cap=200)
    far = np.nonzero((ev.n == 0) & np.isfinite(S64))[0]
    bad = S32.astype(np.float64).copy()
    bad[far[0]] += 1e4 * float(np.float32(float(np.float32(0.9)) ** 40))
    with pytest.raises(AssertionError):
        pc.check_costs(orc, op, p, cmap, params, x0, U, eps, bad, S64, True, 0.0)
    near = np.nonzero(ev.n > 0)[0]
    bad = S32.astype(np.float64).copy()
    k = near[0]
    bad[k] = S_match[k] + 2 * ev.value[k][0] if not ev.on[k][0] else S_match[k] - 2 * ev.value[k][0]
    with pytest.raises(AssertionError):
        pc.check_costs(orc, op, p, cmap, params, x0, U, eps, bad, S64, True, 0.0)
