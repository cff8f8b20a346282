"""The allocation-free entry point (mppi_iterate_noalloc) against the context entry
point it is a variant of (mppi_iterate_device), through the C ABI.

Both run the same kernels with the same launch shape, so the updated controls and
the costs must agree bit for bit (stricter than the 1e-5 bars against the oracle).
Calls follow one another on one stream and share the library's static scratch: a
paper-shaped call (K=1920, T=100, smoothing window 9), then a smaller one (K=256,
T=30, no smoothing, so the tables reload), then the largest the scratch takes
(K=16384 on the schedule with the most blocks, T=256), then the small one again.
"""
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


def _case(M, torch, prob, cmap, params, x0, U0, it, schedule):
    """(U, S, status) from the context path and from the allocation-free path."""
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream()
    sid = int(stream.cuda_stream)
    # context path: mppi_iterate_device from a device x0, iteration counter = it
    with M.Controller(prob, cmap, params, stream=sid, schedule=schedule) as c:
        c.set_controls(U0)
        c.iteration = it
        x_dev = torch.tensor(x0, device=dev)
        M.mppi_iterate_device(c.ctx, x_dev.data_ptr())
        U_ctx, st_ctx = M.mppi_get_controls(c.ctx, prob.T)
        c.set_controls(U0)
        c.iteration = it
        S_ctx, _ = c.iterate(x0, want_costs=True)
    # allocation-free path on caller-owned device buffers
    map_d = torch.from_numpy(np.array(cmap.data, np.float32)).to(dev)
    par_d = torch.from_numpy(np.array(params, np.float32)).to(dev)
    x_d = torch.tensor(x0, device=dev)
    U_d = torch.from_numpy(np.ascontiguousarray(U0, np.float32)).to(dev)
    S_d = torch.full((prob.K,), float("nan"), device=dev)
    st_d = torch.full((1,), -1, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    cfg = M.make_config(prob, schedule=schedule)
    M.mppi_iterate_noalloc(cfg, M.make_cost(prob.cost), 0, sid, map_d.data_ptr(), cmap.data.shape[0],
                           cmap.data.shape[1], cmap.origin_x, cmap.origin_y, cmap.resolution, prob.hidden,
                           par_d.data_ptr(), x_d.data_ptr(), it, U_d.data_ptr(), S_d.data_ptr(), st_d.data_ptr())
    torch.cuda.synchronize()
    return (U_ctx, S_ctx, st_ctx), (U_d.cpu().numpy(), S_d.cpu().numpy(), int(st_d.cpu().item()))


def _check(ctx, na, label):
    U_c, S_c, st_c = ctx
    U_n, S_n, st_n = na
    _say(f"{label}: max |dU| {np.max(np.abs(U_n - U_c)):.3e}  max |dS| {np.nanmax(np.abs(S_n - S_c)):.3e}  "
         f"status {st_n}")
    assert st_n == st_c == 0
    assert np.isfinite(S_n).all()
    np.testing.assert_array_equal(U_n, U_c)
    np.testing.assert_array_equal(S_n, S_c)


def test_noalloc_matches_context_in_turn(env):
    M, torch = env
    ell = synth.ellipse_map()
    ring = synth.ring_map()
    p32 = synth.mlp_params(32, 0)

    big = synth.c2_problem(seed=3)
    U0 = synth.random_controls(big.T, seed=1)
    _say("case: K=1920 T=100 window 9, schedule auto, it=5")
    _check(*_case(M, torch, big, ell, p32, synth.C2_X0, U0, 5, 0), "paper-shaped")

    small = synth.c1_problem(seed=2)
    _say("case: K=256 T=30 window 1, schedule auto, it=0")
    _check(*_case(M, torch, small, ring, p32, synth.C1_X0, np.zeros((small.T, 2), np.float32), 0, 0), "small")

    top = synth.with_(synth.c1_problem(seed=4), K=16384, T=256)
    _say("case: K=16384 T=256 window 1, wave schedule (2048 blocks), it=1")
    _check(*_case(M, torch, top, ring, p32, synth.C1_X0, synth.random_controls(256, seed=2), 1,
                  M.MPPI_SCHED_WAVE), "largest")

    _say("case: K=256 T=30 again, lane schedule, it=9")
    _check(*_case(M, torch, small, ring, p32, synth.C1_X0, synth.random_controls(small.T, seed=3), 9,
                  M.MPPI_SCHED_LANE), "small again")


def test_noalloc_quad_h64_and_null_outputs(env):
    """The matrix-core schedule (h = 64, BF16) with S and the status left to the scratch."""
    M, torch = env
    prob = synth.with_(synth.c3_problem(K=4096, seed=1), T=64)
    cmap = synth.ring_map()
    params = synth.mlp_params(64, 0)
    dev = torch.device("cuda")
    sid = int(torch.cuda.current_stream().cuda_stream)
    U0 = synth.random_controls(prob.T, seed=5)
    with M.Controller(prob, cmap, params, stream=sid, precision=M.MPPI_PREC_BF16) as c:
        c.set_controls(U0)
        c.iteration = 2
        c.iterate(synth.C1_X0)
        U_ctx = c.controls()
    map_d = torch.from_numpy(np.array(cmap.data, np.float32)).to(dev)
    par_d = torch.from_numpy(np.array(params, np.float32)).to(dev)
    x_d = torch.tensor(synth.C1_X0, device=dev)
    U_d = torch.from_numpy(U0.copy()).to(dev)
    cfg = M.make_config(prob, precision=M.MPPI_PREC_BF16)
    _say("case: K=4096 T=64 h=64 BF16 quad, S and status NULL")
    M.mppi_iterate_noalloc(cfg, M.make_cost(prob.cost), 0, sid, map_d.data_ptr(), cmap.data.shape[0],
                           cmap.data.shape[1], cmap.origin_x, cmap.origin_y, cmap.resolution, 64,
                           par_d.data_ptr(), x_d.data_ptr(), 2, U_d.data_ptr())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(U_d.cpu().numpy(), U_ctx)
