"""GPU parity of the basis-function dynamics model (appendix; Section VI-B-1): the HIP
path (lane and wave schedules) against the CPU oracle, with the bars of
parity_checks (samples within 1e-4 of the model's v_x = 0.1 branch point, or of an
impulse threshold, are excluded from the cost comparison)."""
import numpy as np
import pytest

import synth
from parity_checks import check_iteration

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1707_02342_amd import mppi
    mppi.lib()
    return mppi


def _warm(T, seed, throttle=0.3):
    U = synth.random_controls(T, seed, scale=0.2)
    U[:, 1] += throttle
    return U


@pytest.mark.parametrize("schedule", [0, 1, 2])
@pytest.mark.parametrize("seed", [0, 1])
def test_basis_paper_shaped(M, orc, schedule, seed):
    """K=1920, T=100, elliptical 2048^2 map, impulses, SGF 9/2, synthetic Theta."""
    prob = synth.basis_problem(seed)
    print("basis paper-shaped", schedule, seed, flush=True)
    check_iteration(M, orc, prob, synth.ellipse_map(), synth.basis_theta(0), synth.C2_X0,
                    _warm(100, 40 + seed), schedule, it=seed, impulses=True)


@pytest.mark.parametrize("schedule", [1, 2])
@pytest.mark.parametrize("K,T", [(1, 1), (7, 5), (65, 31), (257, 9), (1000, 64), (4100, 12), (300, 200)])
def test_basis_ragged(M, orc, schedule, K, T):
    prob = synth.with_(synth.c1_problem(seed=K + T), K=K, T=T, model=1)
    print("basis ragged", schedule, K, T, flush=True)
    check_iteration(M, orc, prob, synth.ring_map(), synth.basis_theta(1), synth.C1_X0, _warm(T, K),
                    schedule, impulses=True)


@pytest.mark.parametrize("schedule", [1, 2])
def test_basis_low_speed_branch(M, orc, schedule):
    """Starting at v_x = 0.05 with throttle: the first steps take the v_x <= 0.1 branch
    (tan of the steering), later steps the moving branch.  Every sample crosses
    v_x = 0.1 once, so a few (about 0.3 %) pass within 1e-4 of it and are excluded."""
    prob = synth.with_(synth.c1_problem(seed=5), K=512, T=40, model=1)
    x0 = synth.C1_X0.copy()
    x0[4] = 0.05
    U = _warm(40, 5, throttle=0.6)
    op = orc.OracleProblem(prob, synth.ring_map(), synth.basis_theta(2))
    _, tr = orc.rollout(op, x0, U, orc.noise(op, 0), traj=True)
    slow = (tr[:, :-1, 4] <= 0.1).mean()
    print(f"fraction of steps in the low-speed branch {slow:.3f}", flush=True)
    assert 0.005 < slow < 0.5
    check_iteration(M, orc, prob, synth.ring_map(), synth.basis_theta(2), x0, U, schedule, impulses=True,
                    near_cap=0.02)


@pytest.mark.parametrize("schedule", [1, 2])
def test_basis_with_exploration(M, orc, schedule):
    prob = synth.with_(synth.basis_problem(3), K=700, T=50, explore=0.05)
    check_iteration(M, orc, prob, synth.ellipse_map(), synth.basis_theta(0), synth.C2_X0, _warm(50, 3),
                    schedule, impulses=True)


@pytest.mark.parametrize("schedule", [1, 2])
def test_basis_receding_device_loop_matches_host_loop(M, orc, schedule):
    """The fused receding step (shift and plant step in the final block) equals the
    host-driven mppi_iterate + mppi_shift + mppi_plant_step loop bit for bit, and the
    plant step matches the oracle's."""
    prob = synth.with_(synth.basis_problem(4), K=640, T=50)
    cmap, theta = synth.ellipse_map(), synth.basis_theta(0)
    n = 10
    with M.Controller(prob, cmap, theta, schedule=schedule) as c:
        c.set_controls(_warm(50, 9))
        uh, xh, _ = M.mppi_run_receding(c.ctx, synth.C2_X0, n)
    op = orc.OracleProblem(prob, cmap, theta)
    with M.Controller(prob, cmap, theta, schedule=schedule) as c:
        c.set_controls(_warm(50, 9))
        x = synth.C2_X0.copy()
        for i in range(n):
            c.iterate(x)
            u0 = c.shift()
            assert np.array_equal(u0, uh[i])
            xr = orc.plant_step(op, x.astype(np.float64), u0.astype(np.float64))
            x = c.plant_step(x, u0)
            assert np.array_equal(x, xh[i + 1])
            np.testing.assert_allclose(x, xr, rtol=1e-5, atol=1e-5)


def test_basis_rejections(M):
    theta = synth.basis_theta(0)
    prob = synth.with_(synth.c1_problem(), model=1)
    for kw in (dict(schedule=3), dict(schedule=4), dict(precision=M.MPPI_PREC_BF16)):
        with pytest.raises(M.MppiError):
            M.Controller(prob, synth.ring_map(), theta, **kw)
    bad = theta.copy()
    bad[3, 2] = np.nan
    with pytest.raises(M.MppiError):
        M.Controller(prob, synth.ring_map(), bad)
    with M.Controller(synth.with_(prob, K=256, T=20), synth.ring_map(), theta) as c:
        with pytest.raises(M.MppiError):
            c.objective(synth.C1_X0, 0)
        # switching back to the network and to the basis model again
        c.set_dynamics(synth.mlp_params(32, 0))
        c.objective(synth.C1_X0, 0)
        c.set_basis_dynamics(theta)
        c.iterate(synth.C1_X0)
