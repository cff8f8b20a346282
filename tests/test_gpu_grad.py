"""GPU parity of the differentiation form: the free-energy objective
J = -lambda log mean exp(-S/lambda) and its gradient with respect to U and the network
parameters (adjoint rollout with checkpoints) against the oracle's FP64 reverse mode,
which itself is pinned to central finite differences on the CPU.

Bars: J within 1e-5 relative; every gradient entry within
1e-3 * max|g_ref| + 1e-6 of the FP64 oracle (FP32 forward states and a 100-step
reverse accumulation; derivation in the design notes).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

G_RTOL = 1e-3


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1707_02342_amd import mppi
    mppi.lib()
    return mppi


def _grad_check(M, orc, prob, x0, U, it=0, ckpt=10, params=None):
    cmap = synth.ring_map()
    params = synth.mlp_params(32, prob.seed) if params is None else params
    print(f"grad K={prob.K} T={prob.T} seed={prob.seed} ckpt={ckpt}", flush=True)
    with M.Controller(prob, cmap, params) as c:
        c.set_controls(U)
        J, S = c.objective(x0, it, ckpt, want_costs=True)
        gU, gth = c.objective_backward()
        U_after = c.controls()
    assert np.array_equal(U_after, U.astype(np.float32)), "the objective must not update U"
    op = orc.OracleProblem(prob, cmap, params)
    Jr, gUr, gthr = orc.objective_grad(op, x0, U.astype(np.float64), it=it)
    assert abs(J - Jr) <= 1e-5 * max(abs(Jr), 1.0), (J, Jr)
    scale = max(np.abs(gUr).max(), np.abs(gthr).max())
    eU = np.abs(gU - gUr).max()
    eth = np.abs(gth - gthr).max()
    print(f"  J {J:.6f} ref {Jr:.6f}; max|dgU| {eU:.2e} max|dgth| {eth:.2e} scale {scale:.2e}", flush=True)
    assert eU <= G_RTOL * scale + 1e-6
    assert eth <= G_RTOL * scale + 1e-6
    return gU, gth


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_small(M, orc, seed):
    prob = synth.with_(synth.c5_problem(seed=seed), K=64, T=20)
    U = synth.random_controls(20, seed, scale=0.2)
    _grad_check(M, orc, prob, synth.C1_X0, U, it=seed)


@pytest.mark.parametrize("K,T", [(1, 7), (9, 33), (130, 41)])
def test_gradient_ragged(M, orc, K, T):
    prob = synth.with_(synth.c5_problem(seed=3), K=K, T=T)
    _grad_check(M, orc, prob, synth.C1_X0, synth.random_controls(T, K, scale=0.2), ckpt=10)


def test_checkpoint_interval_does_not_change_the_gradient(M, orc):
    prob = synth.with_(synth.c5_problem(seed=4), K=48, T=37)
    U = synth.random_controls(37, 4, scale=0.2)
    ref = None
    for ck in (1, 7, 10, 16):
        gU, gth = _grad_check(M, orc, prob, synth.C1_X0, U, ckpt=ck)
        if ref is None:
            ref = (gU, gth)
        else:
            s = max(np.abs(ref[0]).max(), np.abs(ref[1]).max())
            assert np.abs(gU - ref[0]).max() <= 1e-4 * s
            assert np.abs(gth - ref[1]).max() <= 1e-4 * s


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_gradient_full_size(M, orc, seed):
    """The differentiation workload: K=4096, T=100, checkpoints every 10 steps, seeds 0-4
    (the Philox key, the network and U all follow the seed)."""
    prob = synth.c5_problem(seed=seed)
    _grad_check(M, orc, prob, synth.C1_X0, synth.random_controls(100, seed, scale=0.2), it=seed, ckpt=10)


def test_autograd_function(M, orc):
    import torch
    from paper_1707_02342_amd.autograd import free_energy
    prob = synth.with_(synth.c5_problem(seed=5), K=96, T=24)
    params = synth.mlp_params(32, 5)
    U0 = synth.random_controls(24, 5, scale=0.2)
    with M.Controller(prob, synth.ring_map(), params) as c:
        U = torch.tensor(U0, requires_grad=True)
        th = torch.tensor(params, requires_grad=True)
        J = free_energy(U, th, c, synth.C1_X0, 2)
        J.backward()
        c.set_controls(U0)
        c.set_dynamics(params)
        J2, _ = c.objective(synth.C1_X0, 2)
        gU, gth = c.objective_backward()
    assert float(J) == pytest.approx(J2, rel=1e-12)
    np.testing.assert_array_equal(U.grad.numpy(), gU)
    np.testing.assert_array_equal(th.grad.numpy(), gth)


def test_backward_requires_objective(M):
    prob = synth.with_(synth.c5_problem(), K=16, T=10)
    with M.Controller(prob, synth.ring_map(), synth.mlp_params(32, 0)) as c:
        with pytest.raises(M.MppiError) as e:
            c.objective_backward()
        assert e.value.status == M.MPPI_E_STATE
        c.objective(synth.C1_X0, 0)
        c.objective_backward()
        c.iterate(synth.C1_X0)
        with pytest.raises(M.MppiError):
            c.objective_backward()
        with pytest.raises(M.MppiError):
            c.objective(synth.C1_X0, 0, ckpt_every=17)


def test_adjoint_kernel_timing_slot(M):
    """With timing on, every backward pass records its adjoint rollout kernel in the
    second timing slot; the iteration slot counts the objective's forward launches, and
    the gradient is the same as with timing off."""
    prob = synth.with_(synth.c5_problem(seed=1), K=256, T=40)
    with M.Controller(prob, synth.ring_map(), synth.mlp_params(32, 1)) as c:
        c.set_controls(synth.random_controls(40, 1, scale=0.2))
        c.objective(synth.C1_X0, 0)
        g_off = c.objective_backward()
        M.mppi_set_timing(c.ctx, True)
        for _ in range(3):
            c.objective(synth.C1_X0, 0)
            g_on = c.objective_backward()
        (t0, t1), (n0, n1) = M.mppi_get_timing(c.ctx)
        samples = M.mppi_get_timing_samples(c.ctx)
        M.mppi_set_timing(c.ctx, False)
    assert (n0, n1) == (3, 3)
    assert t0 > 0.0 and t1 > 0.0
    assert len(samples) == 3 and abs(float(np.sum(samples)) - t0) <= 1e-3 * t0
    np.testing.assert_array_equal(g_on[0], g_off[0])
    np.testing.assert_array_equal(g_on[1], g_off[1])
