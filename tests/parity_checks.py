"""Shared parity checks of one MPPI iteration: the HIP path (through the C ABI) against
the CPU oracle on the same seeded inputs.  Test helper, not collected by itself.

Bars (FP32 GPU vs FP64 oracle):
  * S_k: |S_gpu - S_ref| <= 1e-5 * max(|S_ref|, 1); with impulse costs (or the
    basis-function model's speed branch) the samples that pass within 1e-4 of a
    threshold (oracle margin) are excluded and must be fewer than 0.1 %.
  * U, stage-isolated: the oracle's FP64 weights/update applied to the GPU's own S and
    the bit-identical eps reproduces the GPU's U within 1e-5 absolute.
  * U, end to end: GPU U vs the oracle's full iteration within 1e-5 absolute, or
    explained by the first-order sensitivity of the weights to the FP32 cost errors.
"""
import numpy as np

COST_RTOL = 1e-5
U_ATOL = 1e-5


def deltas(prob, eps, U0):
    """delta_{k,t} = v_{k,t} - u_t: eps for samples k < (1 - alpha) K (Algorithm 1's
    importance samples), eps - u_t for the exploration samples after them."""
    d = eps.astype(np.float64).copy()
    alpha = float(np.float32(getattr(prob, "explore", 0.0)))
    zero_mean = ~(np.arange(d.shape[0]) < (1.0 - alpha) * d.shape[0])
    d[zero_mean] -= U0.astype(np.float64)[None]
    return d


def e2e_explained(orc, prob, S_gpu, S_ref, eps, U0, U_gpu, margin=None):
    """End-to-end control difference and its first-order prediction from the cost
    differences dS: d(Delta_t) = -(1/lambda) sum_k w_k (delta_kt - Delta_t)(dS_k - sum_j w_j dS_j),
    smoothed by the SG matrix.  Returns (max|dU|, max|dU - dU_pred|, max|dU_pred|)."""
    S_r = S_ref.copy()
    if margin is not None:
        near = margin < 1e-4
        S_r[near] = S_gpu[near]
    st, w, rho, eta = orc.weights(S_r, prob.lam)
    e64 = deltas(prob, eps, U0)
    delta = np.tensordot(w, e64, axes=(0, 0))
    Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
    U_ref = U0.astype(np.float64) + Mx @ delta
    fin = np.isfinite(S_r) & np.isfinite(S_gpu)
    dS = np.where(fin, S_gpu.astype(np.float64) - np.where(fin, S_r, 0.0), 0.0)
    dSc = dS - np.sum(w * dS)
    dd = -(1.0 / prob.lam) * np.tensordot(w * dSc, e64 - delta[None], axes=(0, 0))
    pred_U = Mx @ dd
    diff = U_gpu.astype(np.float64) - U_ref
    return np.abs(diff).max(), np.abs(diff - pred_U).max(), np.abs(pred_U).max()


def check_iteration(M, orc, prob, cmap, params, x0, U0, schedule, it=0, impulses=False, near_cap=1e-3):
    """One iteration against the oracle; near_cap bounds the fraction of samples that
    pass within 1e-4 of a threshold (excluded from the cost comparison)."""
    with M.Controller(prob, cmap, params, schedule=schedule) as c:
        c.set_controls(U0)
        c.iteration = it
        S, st = c.iterate(x0, want_costs=True)
        Ug = c.controls()
        rho_g, eta_g, delta_g = c.stats()
    op = orc.OracleProblem(prob, cmap, params)
    eps = orc.noise(op, it)
    ref = orc.iterate(op, x0, U0, it)
    assert st == M.MPPI_OK and ref.status == orc.OK
    # S_k: the same samples are non-finite on both sides; finite ones agree to COST_RTOL
    fin = np.isfinite(ref.S)
    assert np.array_equal(np.isfinite(S), fin), "non-finite samples differ"
    Sf = np.where(fin, S.astype(np.float64), 0.0)
    Rf = np.where(fin, ref.S, 0.0)
    err = np.abs(Sf - Rf) / np.maximum(np.abs(Rf), 1.0)
    margin = None
    if impulses:
        margin = orc.threshold_margins(op, x0, U0, eps)
        near = margin < 1e-4
        assert near.mean() < near_cap, near.mean()
        err = np.where(near, 0.0, err)
    worst = int(np.argmax(err))
    assert err.max() <= COST_RTOL, f"S_{worst}: gpu {S[worst]} ref {ref.S[worst]} rel {err.max():.3e}"
    # stage-isolated: oracle weights + update on the GPU's S and the same eps
    st2, w, rho, eta = orc.weights(S.astype(np.float64), prob.lam)
    delta = np.tensordot(w, deltas(prob, eps, U0), axes=(0, 0))
    Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
    U_iso = U0.astype(np.float64) + Mx @ delta
    e_iso = np.abs(Ug - U_iso).max()
    assert e_iso <= U_ATOL, f"stage-isolated |dU| {e_iso:.3e}"
    assert abs(rho_g - rho) <= 1e-6 * max(abs(rho), 1.0)
    np.testing.assert_allclose(delta_g, delta, rtol=0, atol=1e-6)
    # end to end: the difference must be the FP32 cost differences propagated through the
    # exact first-order sensitivity of the weights (samples passing within 1e-4 of an
    # impulse threshold take the GPU's cost on the oracle side too)
    e2e, resid, pred = e2e_explained(orc, prob, S, ref.S, eps, U0, Ug,
                                     margin if impulses else None)
    print(f"K={prob.K} T={prob.T} sched={schedule}: max rel dS {err.max():.2e}, |dU| iso {e_iso:.2e} "
         f"e2e {e2e:.2e} predicted {pred:.2e} residual {resid:.2e}", flush=True)
    assert resid <= 2e-6 + 0.05 * pred + e_iso, f"end-to-end |dU| {e2e:.3e} not explained (residual {resid:.3e})"
    assert e2e <= U_ATOL or e2e <= 1.1 * pred + e_iso + 2e-6
    return S, Ug


def check_cem(M, orc, prob, cmap, params, x0, U0, schedule, it=0, impulses=False):
    """One iteration with Algorithm 3's weights against the oracle (the bars of the CEM
    parity tests: costs, the stage-isolated elite average, and the end-to-end swap)."""
    with M.Controller(prob, cmap, params, schedule=schedule) as c:
        c.set_controls(U0)
        c.iteration = it
        S, st = c.iterate(x0, want_costs=True)
        Ug = c.controls()
        z_g, n_g, delta_g = c.stats()
    op = orc.OracleProblem(prob, cmap, params)
    eps = orc.noise(op, it)
    ref = orc.iterate(op, x0, U0, it)
    zeta = orc.cem_zeta(prob.K, prob.elite)
    assert st == M.MPPI_OK and ref.status == orc.OK
    fin = np.isfinite(ref.S)
    assert np.array_equal(np.isfinite(S), fin), "non-finite samples differ"
    Sf, Rf = np.where(fin, S.astype(np.float64), 0.0), np.where(fin, ref.S, 0.0)
    err = np.abs(Sf - Rf) / np.maximum(np.abs(Rf), 1.0)
    if impulses:
        margin = orc.threshold_margins(op, x0, U0, eps)
        near = margin < 1e-4
        assert near.mean() < 1e-3
        err = np.where(near, 0.0, err)
    assert err.max() <= COST_RTOL, f"max rel dS {err.max():.3e}"
    d = deltas(prob, eps, U0)
    Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
    # stage-isolated: the oracle's Algorithm 3 on the GPU's costs
    st2, w_iso, z_iso, n_iso = orc.weights_cem(S.astype(np.float64), zeta)
    delta_iso = np.tensordot(w_iso, d, axes=(0, 0))
    e_iso = np.abs(Ug - (U0.astype(np.float64) + Mx @ delta_iso)).max()
    assert e_iso <= U_ATOL, f"stage-isolated |dU| {e_iso:.3e}"
    np.testing.assert_allclose(delta_g, delta_iso, rtol=0, atol=1e-6)
    assert n_g == n_iso and z_g == np.float32(z_iso), (n_g, n_iso, z_g, z_iso)
    # end to end: the two elite sets differ only at the threshold, and U by that swap
    E_g, E_r = set(np.nonzero(w_iso)[0]), set(np.nonzero(ref.w)[0])
    swapped = sorted(E_g ^ E_r)
    z_r = ref.rho
    for k in swapped:
        assert abs(ref.S[k] - z_r) <= 1e-5 * max(abs(z_r), 1.0), (k, ref.S[k], z_r)
    pred = Mx @ ((d[sorted(E_g - E_r)].sum(axis=0) - d[sorted(E_r - E_g)].sum(axis=0)) / n_iso) if swapped else 0.0
    resid = np.abs(Ug - ref.U - pred).max()
    print(f"CEM K={prob.K} T={prob.T} sched={schedule} zeta={zeta}: rel dS {err.max():.2e}, |dU| iso "
         f"{e_iso:.2e}, swapped {len(swapped)}, e2e residual {resid:.2e}", flush=True)
    assert resid <= U_ATOL
    return S, Ug
