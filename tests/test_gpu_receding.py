"""Receding-horizon steps on device data: mppi_run_receding_device (one multi-step
cooperative launch where the wave schedule's split form applies, else one launch per
step) against the same number of mppi_step_device calls, bit for bit: U, the plant
state, the u_0 and state histories, the costs of the last step and the iteration
counter; a multi-step launch followed by single steps continues the same sequence.

The oracle parity of the paper-shaped receding loop itself is tested in
test_gpu_parity.py (test_receding_horizon_loop), which runs mppi_run_receding, itself
one multi-step launch on that workload."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1707_02342_amd import mppi
    mppi.lib()
    return mppi, torch


def _say(*a):
    print(*a, flush=True)


def _run(M, torch, prob, cmap, params, x0, U0, n, multi, split_after=None, schedule=0):
    """(U, x, u_hist, x_hist, iteration) after n receding steps, either through
    mppi_run_receding_device (multi) or n mppi_step_device calls."""
    dev = torch.device("cuda")
    with M.Controller(prob, cmap, params, schedule=schedule) as c:
        c.set_controls(U0)
        c.iteration = 3
        x = torch.tensor(x0, device=dev)
        uh = torch.full((max(n, 1), 2), float("nan"), device=dev)
        xh = torch.full((max(n, 1), 7), float("nan"), device=dev)
        if multi:
            m = n if split_after is None else split_after
            M.mppi_run_receding_device(c.ctx, x.data_ptr(), m, uh.data_ptr(), xh.data_ptr())
            for i in range(m, n):
                M.mppi_step_device(c.ctx, x.data_ptr(), uh[i].data_ptr())
                xh[i].copy_(x)
        else:
            for i in range(n):
                M.mppi_step_device(c.ctx, x.data_ptr(), uh[i].data_ptr())
                xh[i].copy_(x)
        torch.cuda.synchronize()
        U, st = M.mppi_get_controls(c.ctx, prob.T)
        assert st == M.MPPI_OK
        return U, x.cpu().numpy(), uh.cpu().numpy()[:n], xh.cpu().numpy()[:n], c.iteration, c.schedule


@pytest.mark.parametrize("n", [1, 2, 37])
def test_multi_step_equals_single_steps_paper_shaped(env, n):
    M, torch = env
    prob = synth.c2_problem(seed=2)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    U0 = synth.random_controls(prob.T, 4, scale=0.2)
    _say(f"case: paper-shaped, {n} steps")
    a = _run(M, torch, prob, cmap, params, synth.C2_X0, U0, n, True)
    b = _run(M, torch, prob, cmap, params, synth.C2_X0, U0, n, False)
    for x, y in zip(a[:4], b[:4]):
        np.testing.assert_array_equal(x, y)
    assert a[4] == b[4] == 3 + n


def test_multi_step_then_single_steps(env):
    """A multi-step launch of 20 steps, then 5 single steps, equals 25 single steps (the
    iteration counter and the signal words' step numbering carry over)."""
    M, torch = env
    prob = synth.c2_problem(seed=3)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    U0 = np.zeros((prob.T, 2), np.float32)
    a = _run(M, torch, prob, cmap, params, synth.C2_X0, U0, 25, True, split_after=20)
    b = _run(M, torch, prob, cmap, params, synth.C2_X0, U0, 25, False)
    for x, y in zip(a[:4], b[:4]):
        np.testing.assert_array_equal(x, y)


def test_multi_step_repeated_launches(env):
    """Three multi-step launches on one context in a row equal the single-step sequence."""
    M, torch = env
    prob = synth.c2_problem(seed=4)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    dev = torch.device("cuda")
    res = []
    for multi in (True, False):
        with M.Controller(prob, cmap, params) as c:
            x = torch.tensor(synth.C2_X0, device=dev)
            if multi:
                for n in (10, 1, 15):
                    M.mppi_run_receding_device(c.ctx, x.data_ptr(), n)
            else:
                for _ in range(26):
                    M.mppi_step_device(c.ctx, x.data_ptr())
            torch.cuda.synchronize()
            res.append((c.controls(), x.cpu().numpy(), c.iteration))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2] == 26


@pytest.mark.parametrize("case", ["basis", "exploration", "K_over_cus", "T_over_128", "lane"])
def test_multi_step_other_forms(env, case):
    """The basis-function model and exploration samples in the multi-step launch, and the
    per-step fallback (more blocks than compute units, T > 128, another schedule)."""
    M, torch = env
    cmap = synth.ellipse_map()
    x0 = synth.C2_X0
    if case == "basis":
        prob = synth.basis_problem(seed=1)
        params = synth.basis_theta(0)
        x0 = synth.ellipse_pose(0.0, 4.0)
    elif case == "exploration":
        prob = synth.explore_problem(seed=1)
        params = synth.mlp_params(32, 0)
    elif case == "K_over_cus":
        prob = synth.with_(synth.c2_problem(seed=1), K=4100)
        params = synth.mlp_params(32, 0)
    elif case == "T_over_128":
        prob = synth.with_(synth.c2_problem(seed=1), K=512, T=160)
        params = synth.mlp_params(32, 0)
    else:
        prob = synth.with_(synth.c2_problem(seed=1), K=512)
        params = synth.mlp_params(32, 0)
    U0 = synth.random_controls(prob.T, 6, scale=0.1)
    if case == "basis":
        U0[:, 1] = 0.3
    _say(f"case: {case}")
    sched = M.MPPI_SCHED_LANE if case == "lane" else 0
    a = _run(M, torch, prob, cmap, params, x0, U0, 6, True, schedule=sched)
    b = _run(M, torch, prob, cmap, params, x0, U0, 6, False, schedule=sched)
    for x, y in zip(a[:4], b[:4]):
        np.testing.assert_array_equal(x, y)
    assert np.isfinite(a[0]).all()


def test_run_receding_device_rejects_bad_arguments(env):
    M, torch = env
    prob = synth.c1_problem()
    with M.Controller(prob, synth.ring_map(), synth.mlp_params(32, 0)) as c:
        with pytest.raises(M.MppiError):
            M.mppi_run_receding_device(c.ctx, 0, 3)
        x = torch.tensor(synth.C1_X0, device="cuda")
        with pytest.raises(M.MppiError):
            M.mppi_run_receding_device(c.ctx, x.data_ptr(), -1)
        M.mppi_run_receding_device(c.ctx, x.data_ptr(), 0)


def test_multi_step_give_up_then_recover(env, monkeypatch):
    """A multi-step launch whose blocks may poll another block's signal only once gives up
    (the bound of the kernel's own wait, set from the host): the next synchronising call
    reports MPPI_E_DEVICE.  The same context, reset to the start state, then runs a normal
    launch that equals a fresh context's: the signal words the aborted launch left hold
    steps below the next launch's."""
    M, torch = env
    prob = synth.c2_problem(seed=6)
    cmap, params = synth.ellipse_map(), synth.mlp_params(32, 0)
    with M.Controller(prob, cmap, params) as c:
        x = torch.tensor(synth.C2_X0, device="cuda")
        monkeypatch.setenv("MPPI_STEP_SPIN_LIMIT", "1")
        M.mppi_run_receding_device(c.ctx, x.data_ptr(), 8)
        monkeypatch.delenv("MPPI_STEP_SPIN_LIMIT")
        with pytest.raises(M.MppiError):
            M.mppi_get_controls(c.ctx, prob.T)
        c.set_controls(np.zeros((prob.T, 2), np.float32))
        c.iteration = 0
        got = _run_once(M, torch, c, prob, 8)
    with M.Controller(prob, cmap, params) as fresh:
        ref = _run_once(M, torch, fresh, prob, 8)
    for a_, b_ in zip(got, ref):
        np.testing.assert_array_equal(a_, b_)


def _run_once(M, torch, c, prob, n):
    x = torch.tensor(synth.C2_X0, device="cuda")
    M.mppi_run_receding_device(c.ctx, x.data_ptr(), n)
    torch.cuda.synchronize()
    U, st = M.mppi_get_controls(c.ctx, prob.T)
    assert st == M.MPPI_OK
    return U, x.cpu().numpy()
