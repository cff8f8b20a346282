"""Closed-loop lap harness on the GPU: the cost-map lookup used to classify laps
against the oracle's cost map, and short lap runs of the IT and CEM controllers with the
basis-function plant at the parameter table's settings."""
import numpy as np
import pytest

import synth
from parity_checks import check_cem, check_iteration

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1707_02342_amd import mppi
    mppi.lib()
    return mppi


def test_costmap_values_match_the_oracle(M, orc):
    prob = synth.c2_problem(0)
    cmap = synth.ellipse_map()
    rng = np.random.default_rng(0)
    xy = np.concatenate([rng.uniform(-5.0, 110.0, size=(4000, 2)),
                         synth.ellipse_pose(0.7, 5.0)[None, :2]]).astype(np.float32)
    with M.Controller(prob, cmap, synth.mlp_params(32, 0)) as c:
        h = M.mppi_costmap_values(c.ctx, xy)
        with pytest.raises(M.MppiError):
            M.mppi_costmap_values(c.ctx, np.array([[np.nan, 1.0]], np.float32))
    op = orc.OracleProblem(prob, cmap, synth.mlp_params(32, 0))
    ref = np.array([orc.costmap(op, float(x), float(y))[0] for x, y in xy])
    np.testing.assert_allclose(h, ref, rtol=0, atol=2e-6)


@pytest.mark.parametrize("weighting", [0, 1])
@pytest.mark.parametrize("direction", [1, -1])
def test_lap_runs(M, weighting, direction):
    from paper_1707_02342_amd import laps
    prob = synth.with_(synth.explore_problem(0), model=1, weighting=weighting, elite=0.8)
    x0 = synth.ellipse_pose(0.0, 4.0)
    if direction < 0:
        x0[2] += np.pi
    with M.Controller(prob, synth.ellipse_map(), synth.basis_theta(0)) as c:
        m = laps.evaluate(c, x0, 3, prob.dt, laps.Track(), direction, prob.cost.map_thresh, max_steps=20000)
    print({k: v for k, v in m.items() if k != "per_lap"}, flush=True)
    assert m["laps"] == 2 and m["success_pct"] == 100.0
    assert 15.0 < m["lap_time_mean"] < 120.0
    assert 0.0 < m["speed_min"] <= m["speed_max"] < 20.0


@pytest.mark.parametrize("weighting", [0, 1])
def test_closed_loop_steps_match_the_oracle(M, orc, weighting):
    """The lap runs' configuration (basis-function plant, parameter table, 1 % exploration)
    driven step by step from the host: every fifth step's iteration is checked against
    the oracle from that step's own state, controls and iteration counter, and the
    device-resident loop reproduces the host loop bit for bit."""
    prob = synth.with_(synth.explore_problem(0), model=1, weighting=weighting, elite=0.8)
    cmap, theta = synth.ellipse_map(), synth.basis_theta(0)
    op = orc.OracleProblem(prob, cmap, theta)
    x = synth.ellipse_pose(0.0, 4.0)
    n = 20
    xs, us = [x.copy()], []
    with M.Controller(prob, cmap, theta) as c:
        for i in range(n):
            U_in = c.controls()
            if i % 5 == 0:
                check = check_cem if weighting else check_iteration
                check(M, orc, prob, cmap, theta, x, U_in, c.schedule, it=i, impulses=True)
            c.iterate(x)
            u0 = c.shift()
            xr = orc.plant_step(op, x.astype(np.float64), u0.astype(np.float64))
            x = c.plant_step(x, u0)
            np.testing.assert_allclose(x, xr, rtol=1e-5, atol=1e-5)
            us.append(u0)
            xs.append(x.copy())
    with M.Controller(prob, cmap, theta) as c:
        uh, xh, _ = M.mppi_run_receding(c.ctx, xs[0], n)
    assert np.array_equal(uh, np.array(us)) and np.array_equal(xh, np.array(xs))
