"""Pins of the oracle's vehicle model and state cost (Section VI-B, VI-C).

* Network shape: the paper's 1412 parameters; forward pass against PyTorch (CPU, fp64).
* Kinematics: with the network's output layer zeroed, the dynamic states are constant
  and the explicit-Euler kinematics have closed forms (straight line, discrete arc);
  with a constant output bias the speed grows linearly.
* Cost: constant and affine maps (bilinear interpolation reproduces affine data
  exactly), clamp-to-edge, impulse thresholds just either side, slip angle.
"""
import math

import numpy as np
import pytest
import torch

import synth

ROOT = __import__("pathlib").Path(__file__).resolve().parent


def _golden(name):
    out = {}
    for line in (ROOT / "golden" / name).read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            key, *vals = line.split()
            out[key] = vals
    return out


def test_param_count_matches_paper():
    g = _golden("nn_param_count.txt")
    assert synth.mlp_param_count(int(g["hidden"][0])) == int(g["params"][0])
    assert synth.mlp_params(32, 0).size == 1412


@pytest.mark.parametrize("hidden", [32, 64])
def test_mlp_forward_against_torch(orc, hidden):
    params = synth.mlp_params(hidden, seed=3, bias_scale=0.2)
    p = synth.with_(synth.c1_problem(), hidden=hidden)
    op = orc.OracleProblem(p, synth.constant_map(0.0), params)
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a, dtype=torch.float64) for a in synth.mlp_unpack(params, hidden)]
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.normal(size=6)
        xt = torch.tensor(x)
        ref = torch.nn.functional.linear(
            torch.tanh(torch.nn.functional.linear(torch.tanh(torch.nn.functional.linear(xt, W1, b1)), W2, b2)),
            W3, b3).numpy()
        np.testing.assert_allclose(orc.mlp_forward(op, x), ref, rtol=1e-13, atol=1e-14)


def _zero_output(params, hidden, b3=(0, 0, 0, 0)):
    params = params.copy()
    n_before = 6 * hidden + hidden + hidden * hidden + hidden
    params[n_before:n_before + 4 * hidden] = 0.0
    params[-4:] = np.float32(b3)
    return params


def test_kinematics_closed_form_arc(orc):
    """W3 = 0, b3 = 0: x_d constant; theta_t = theta_0 + t dt w and
    p_t = p_0 + dt sum_{s<t} Rot(theta_s) [v_x, v_y] (a discrete arc, geometric sum)."""
    hidden, T, dt = 32, 40, 0.02
    params = _zero_output(synth.mlp_params(hidden, 0), hidden)
    p = synth.with_(synth.c1_problem(), K=3, T=T, dt=dt)
    op = orc.OracleProblem(p, synth.constant_map(0.0, H=8, W=8), params)
    x0 = np.array([1.5, -2.0, 0.3, 0.1, 3.0, 0.5, 0.7], dtype=np.float32)
    U = np.zeros((T, 2), np.float32)
    eps = orc.noise(op, 0)
    _, tr = orc.rollout(op, x0, U, eps, traj=True)
    x0d = x0.astype(np.float64)
    dt = float(np.float32(dt))                 # parameters enter as fp32
    w, th0, vx, vy = x0d[6], x0d[2], x0d[4], x0d[5]
    for t in range(T + 1):
        th = th0 + t * dt * w
        # sum_{s<t} exp(i(th0 + s dt w)) = exp(i th0) (1 - exp(i t dt w)) / (1 - exp(i dt w))
        g = np.exp(1j * th0) * (1 - np.exp(1j * t * dt * w)) / (1 - np.exp(1j * dt * w))
        vel = vx + 1j * vy
        pos = x0d[0] + 1j * x0d[1] + dt * g * vel
        for k in range(3):
            np.testing.assert_allclose(tr[k, t, 2], th, rtol=0, atol=1e-12)
            np.testing.assert_allclose(tr[k, t, 0] + 1j * tr[k, t, 1], pos, rtol=0, atol=1e-11)
            np.testing.assert_allclose(tr[k, t, 3:], x0d[3:], rtol=0, atol=0)


def test_kinematics_straight_line_and_acceleration(orc):
    """W3 = 0, b3 = (0, a, 0, 0), theta_dot = 0: v_x(t) = v0 + a t dt,
    p_x(t) = p0 + dt cos(theta0) sum_{s<t} v_x(s)."""
    hidden, T, dt, a = 32, 25, 0.02, 1.5
    params = _zero_output(synth.mlp_params(hidden, 1), hidden, b3=(0.0, a, 0.0, 0.0))
    p = synth.with_(synth.c1_problem(), K=2, T=T, dt=dt)
    op = orc.OracleProblem(p, synth.constant_map(0.0, H=8, W=8), params)
    x0 = np.array([0.0, 0.0, 0.0, 0.0, 2.0, 0.0, 0.0], dtype=np.float32)
    eps = orc.noise(op, 0)
    _, tr = orc.rollout(op, x0, np.zeros((T, 2), np.float32), eps, traj=True)
    a64 = float(np.float32(a))
    dt64 = float(np.float32(dt))
    for t in range(T + 1):
        vx = 2.0 + a64 * t * dt64
        px = dt64 * sum(2.0 + a64 * s * dt64 for s in range(t))
        assert abs(tr[0, t, 4] - vx) < 1e-12
        assert abs(tr[0, t, 0] - px) < 1e-12
        assert tr[0, t, 1] == 0.0


def test_constant_map_cost_closed_form(orc):
    """Constant map h = c0, zero network output: per step 100 c0 + (v_x - 6)^2, plus the
    control term gamma sum_i u_i eps_i / Sigma_ii; summed over t = 1..T."""
    hidden, T = 32, 12
    c0 = 0.37
    params = _zero_output(synth.mlp_params(hidden, 0), hidden)
    p = synth.with_(synth.c1_problem(), K=5, T=T, lam=2.0)
    cm = synth.constant_map(c0, H=16, W=16)
    op = orc.OracleProblem(p, cm, params)
    x0 = np.array([2.0, 3.0, 0.4, 0.0, 4.5, 0.0, 0.0], dtype=np.float32)
    U = synth.random_controls(T, 0)
    eps = orc.noise(op, 0)
    S = orc.rollout(op, x0, U, eps)
    c0f = float(np.float32(c0))
    for k in range(5):
        ref = T * (100.0 * c0f + (4.5 - 6.0) ** 2)
        s2 = np.float32(p.sigma2).astype(np.float64)
        ref += 2.0 * np.sum(U.astype(np.float64) * eps[k].astype(np.float64) / s2)
        assert abs(S[k] - ref) < 1e-9 * abs(ref)


def test_bilinear_exact_on_affine_map(orc):
    a, b, c = 0.25, 0.0125, -0.0075
    cm = synth.affine_map(a, b, c, H=40, W=50, resolution=0.5, origin=(-3.0, 2.0))
    op = orc.OracleProblem(synth.c1_problem(), cm, synth.mlp_params(32, 0))
    rng = np.random.default_rng(4)
    for _ in range(200):
        gx, gy = rng.uniform(0, 49), rng.uniform(0, 39)
        px, py = -3.0 + gx * 0.5, 2.0 + gy * 0.5
        h, grad = orc.costmap(op, px, py)
        assert abs(h - (a + b * gy + c * gx)) < 2e-6      # map stored in fp32
        np.testing.assert_allclose(grad, [c / 0.5, b / 0.5], rtol=1e-3, atol=1e-6)


def test_bilinear_grid_points_and_clamp_to_edge(orc):
    rng = np.random.default_rng(5)
    data = rng.uniform(0, 1, size=(6, 9)).astype(np.float32)
    cm = synth.CostMap(data, 1.0, -2.0, 0.25)
    op = orc.OracleProblem(synth.c1_problem(), cm, synth.mlp_params(32, 0))
    for i in range(6):
        for j in range(9):
            assert orc.costmap(op, 1.0 + 0.25 * j, -2.0 + 0.25 * i)[0] == pytest.approx(float(data[i, j]), abs=1e-15)
    # beyond the map the edge value is held
    assert orc.costmap(op, -50.0, -2.0)[0] == pytest.approx(float(data[0, 0]), abs=1e-15)
    assert orc.costmap(op, 1.0 + 0.25 * 8 + 7.0, -2.0 + 0.25 * 5 + 9.0)[0] == pytest.approx(float(data[5, 8]), abs=1e-15)
    assert orc.costmap(op, 1.0 + 0.25 * 3, 1e9)[0] == pytest.approx(float(data[5, 3]), abs=1e-15)
    assert math.isnan(orc.costmap(op, float("nan"), 0.0)[0])


def test_impulse_thresholds_and_slip(orc):
    """Track impulse 1e4*0.9^t*[h > 0.99]; slip zeta = -atan2(v_y, |v_x|), quadratic plus
    impulse 1e4*[|zeta| > 0.75] (Section VI-C)."""
    p = synth.c2_problem()
    for hval, t in ((0.99 - 1e-6, 3), (0.99 + 1e-6, 3), (0.995, 1), (0.995, 50)):
        cm = synth.constant_map(hval)
        op = orc.OracleProblem(p, cm, synth.mlp_params(32, 0))
        x = [5.0, 5.0, 0.0, 0.0, 8.0, 0.0, 0.0]
        c, _ = orc.state_cost(op, x, t)
        hf = float(np.float32(hval))
        decay = float(np.float32(float(np.float32(0.9)) ** t))     # fl32(0.9f^t), parameters enter as fp32
        expect = 100.0 * hf + (1e4 * decay if hf > float(np.float32(0.99)) else 0.0)
        assert c == pytest.approx(expect, rel=1e-12)
    op = orc.OracleProblem(p, synth.constant_map(0.0), synth.mlp_params(32, 0))
    for vx, vy in ((8.0, 0.5), (-8.0, 0.5), (3.0, -2.0), (1.0, 1.0), (0.0, 0.0)):
        zeta = -math.atan2(vy, abs(vx))
        c, g = orc.state_cost(op, [5.0, 5.0, 0.0, 0.0, vx, vy, 0.0], 1)
        expect = (vx - 8.0) ** 2 + zeta ** 2 + (1e4 if abs(zeta) > float(np.float32(0.75)) else 0.0)
        assert c == pytest.approx(expect, rel=1e-12, abs=1e-12)
    # gradient of the smooth part against central differences
    x = np.array([5.0, 5.0, 0.0, 0.0, 6.5, 0.7, 0.0])
    c, g = orc.state_cost(op, x, 1)
    for i in (4, 5):
        d = np.zeros(7)
        d[i] = 1e-6
        fd = (orc.state_cost(op, x + d, 1)[0] - orc.state_cost(op, x - d, 1)[0]) / 2e-6
        assert g[i] == pytest.approx(fd, rel=1e-6)


def test_fp32_and_fp64_oracles_agree(orc):
    """Self-consistency: the FP32 instantiation of the same rollout stays within the
    FP32 error scale of the FP64 one on the small ring-track workload."""
    p = synth.c1_problem()
    op = orc.OracleProblem(p, synth.ring_map(), synth.mlp_params(32, 0))
    eps = orc.noise(op, 0)
    U = synth.random_controls(p.T, 1)
    S64 = orc.rollout(op, synth.C1_X0, U, eps)
    S32 = orc.rollout(op, synth.C1_X0, U, eps, precision="f32")
    rel = np.abs(S32 - S64) / np.maximum(np.abs(S64), 1.0)
    assert rel.max() < 1e-5, rel.max()
