"""Shared parity checks of one MPPI iteration: the HIP path (through the C ABI) against
the CPU oracle on the same seeded inputs.  Test helper, not collected by itself.

Bars (FP32 GPU vs FP64 oracle):
  * S_k: |S_gpu - S_match| <= 1e-5 * max(|S_match|, 1) for EVERY finite sample.  S_match is
    the oracle's cost, except where the oracle's trajectory decides an impulse indicator
    (crash or slip term, Section VI-C) within 1e-4 of its threshold: there the FP32
    trajectory may take either side, so the oracle lists every such term
    (orc_threshold_events) and S_match is the oracle-side cost with the subset of those
    terms that the GPU's S is nearest to (the FP32 trajectory differs from the FP64 one
    by rounding only; the indicators do not feed back into it).  Nothing is excluded,
    and no GPU value enters the reference.  The basis-function model alone also branches
    in its dynamics (v_x > 0.1); samples whose FP64 trajectory passes within 1e-4 of that
    branch point diverge legitimately and are left out (their share is capped per test).
  * U, stage-isolated (hard gate): the oracle's FP64 weights/update applied to the GPU's
    own S and the bit-identical eps reproduce the GPU's U within 1e-5 absolute.
  * U, end to end: |U_gpu - U_ref| where U_ref is the oracle's update from S_match.  It
    must be <= 1e-5, or within the rigorous bound that the measured cost differences
    dS = S_gpu - S_match imply: every weight moves by at most a factor e^{2A},
    A = (max dS - min dS) / (2 lambda), so |dDelta_t| <= (e^{2A} - 1) sum_k w_k |delta_kt - Delta_t|,
    smoothed by |SG|.  Both numbers, the bound that the 1e-5 cost bar itself allows, and
    the first-order prediction from dS are written to the parity record.
"""
import json
import os
from dataclasses import replace
from pathlib import Path

import numpy as np

COST_RTOL = 1e-5
U_ATOL = 1e-5
NEAR_WINDOW = 1e-4

# Per-check records (one dict per checked iteration), written out by the test session
# (conftest.py) to the file named by MPPI_PARITY_RECORD, or test_records/parity_records.jsonl.
RECORDS = []
CURRENT_TEST = {"id": None}


def record(**fields):
    rec = {"test": CURRENT_TEST["id"]}
    for k, v in fields.items():
        if isinstance(v, (np.floating, np.integer)):
            v = v.item()
        rec[k] = v
    RECORDS.append(rec)


def _compact(v):
    """Floats to 4 significant digits (the records are read by eye and kept small)."""
    if isinstance(v, float) and np.isfinite(v):
        return float(f"{v:.4g}")
    return v


SUMMARY_FIELDS = ("max_rel_dS", "dU_iso", "dU_e2e", "dU_e2e_bound", "n_near_threshold", "n_other_side",
                  "n_branch_excluded")


def summary_markdown(records) -> str:
    """Per test function (all its parameter sets) and check: the number of checked
    iterations, their shapes, and the largest value of every field in SUMMARY_FIELDS."""
    groups = {}
    for r in records:
        test = (r.get("test") or "").split("[")[0]
        groups.setdefault((test, r.get("check")), []).append(r)
    lines = ["| test | check | n | K | T | " + " | ".join(SUMMARY_FIELDS) + " |",
             "|---|---|---|---|---|" + "---|" * len(SUMMARY_FIELDS)]
    for (test, check), rs in groups.items():
        cells = []
        for f in SUMMARY_FIELDS:
            vals = [r[f] for r in rs if isinstance(r.get(f), (int, float))]
            cells.append(f"{max(vals):.3g}" if vals else "")
        Ks = sorted({r.get("K") for r in rs if r.get("K") is not None})
        Ts = sorted({r.get("T") for r in rs if r.get("T") is not None})
        lines.append(f"| {test} | {check} | {len(rs)} | {','.join(map(str, Ks))} | {','.join(map(str, Ts))} | "
                     + " | ".join(cells) + " |")
    return "\n".join(lines) + "\n"


def write_records(root: Path):
    """Appends this session's records to MPPI_PARITY_RECORD (default: the repository's
    test_records/parity_records.jsonl) and writes beside it their per-test summary
    (parity_summary.md) and the precision form's records (precision_errors.jsonl)."""
    if not RECORDS:
        return None
    path = Path(os.environ.get("MPPI_PARITY_RECORD", root / "test_records" / "parity_records.jsonl"))
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "a") as f:
        for r in RECORDS:
            f.write(json.dumps({k: _compact(v) for k, v in r.items()}) + "\n")
    (path.parent / "parity_summary.md").write_text(summary_markdown(RECORDS))
    prec = [r for r in RECORDS if r.get("check") == "precision"]
    if prec:
        with open(path.parent / "precision_errors.jsonl", "w") as f:
            for r in prec:
                f.write(json.dumps({k: _compact(v) for k, v in r.items()}) + "\n")
    return path


def deltas(prob, eps, U0):
    """delta_{k,t} = v_{k,t} - u_t: eps for samples k < (1 - alpha) K (Algorithm 1's
    importance samples), eps - u_t for the exploration samples after them."""
    d = eps.astype(np.float64).copy()
    alpha = float(np.float32(getattr(prob, "explore", 0.0)))
    zero_mean = ~(np.arange(d.shape[0]) < (1.0 - alpha) * d.shape[0])
    d[zero_mean] -= U0.astype(np.float64)[None]
    return d


def match_costs(S_gpu, S_ref, events, rtol=COST_RTOL):
    """The oracle-side cost each GPU cost must equal.  For a sample without near-threshold
    terms that is S_ref; otherwise the candidate S_ref - (taken terms) + (a subset of the
    listed terms) nearest to S_gpu.  Returns (S_match, near, flipped): near marks samples
    with listed terms, flipped those whose matched subset differs from the oracle's own."""
    S_match = np.asarray(S_ref, np.float64).copy()
    K = S_match.size
    near = np.zeros(K, bool)
    flipped = np.zeros(K, bool)
    if events is None:
        return S_match, near, flipped
    for k in np.nonzero(events.n > 0)[0]:
        near[k] = True
        if not np.isfinite(S_match[k]) or not np.isfinite(S_gpu[k]):
            continue
        vals, on = events.value[k], events.on[k].astype(bool)
        base = S_match[k] - np.sum(vals[on])
        uniq, counts = np.unique(vals, return_counts=True)
        assert np.prod(counts + 1.0) <= 1 << 22, f"sample {k}: too many near-threshold terms to enumerate"
        sums = np.zeros(1)
        for u, c in zip(uniq, counts):
            sums = (sums[:, None] + u * np.arange(c + 1)[None, :]).ravel()
        cand = base + sums
        j = int(np.argmin(np.abs(cand - float(S_gpu[k]))))
        if abs(cand[j] - S_match[k]) > 0.5 * uniq.min():
            flipped[k] = True
            S_match[k] = cand[j]
    return S_match, near, flipped


def _events(orc, op, prob, x0, U0, eps):
    return orc.threshold_events(op, x0, U0, eps, window=NEAR_WINDOW, cap=max(64, 2 * prob.T))


def branch_margins(orc, prob, cmap, params, x0, U0, eps):
    """Basis-function model: per sample, the smallest |v_x - 0.1| over the states entering
    each step (the model's branch point), from the oracle with the cost thresholds off."""
    cost = replace(prob.cost, map_thresh=float("inf"), slip_thresh=float("inf"))
    op = orc.OracleProblem(replace(prob, cost=cost), cmap, params)
    return orc.threshold_margins(op, x0, U0, eps)


def e2e_bounds(prob, S_match, S_gpu, d, w, delta, Mx):
    """(measured, allowed): the rigorous bounds on the end-to-end |dU| implied by the
    measured cost differences, and by cost differences anywhere within the 1e-5 bar."""
    fin = np.isfinite(S_match) & np.isfinite(S_gpu)
    B = np.tensordot(w, np.abs(d - delta[None]), axes=(0, 0))        # [T][2]
    aM = np.abs(Mx)
    out = []
    dS = (S_gpu.astype(np.float64) - S_match)[fin] / prob.lam
    A = 0.5 * (dS.max() - dS.min()) if dS.size else 0.0
    out.append(float(np.max(aM @ (np.expm1(2.0 * A) * B))))
    tol = COST_RTOL * np.maximum(np.abs(S_match[fin]), 1.0) / prob.lam
    A_tol = float(tol.max()) if tol.size else 0.0
    out.append(float(np.max(aM @ (np.expm1(2.0 * A_tol) * B))))
    return out


def first_order(prob, S_match, S_gpu, d, w, delta, Mx):
    """First-order prediction of U_gpu - U_ref from the cost differences:
    dDelta_t = -(1/lambda) sum_k w_k (delta_kt - Delta_t)(dS_k - sum_j w_j dS_j), smoothed."""
    fin = np.isfinite(S_match) & np.isfinite(S_gpu)
    dS = np.where(fin, S_gpu.astype(np.float64) - np.where(fin, S_match, 0.0), 0.0)
    dSc = dS - np.sum(w * dS)
    dd = -(1.0 / prob.lam) * np.tensordot(w * dSc, d - delta[None], axes=(0, 0))
    return Mx @ dd


def end_to_end(orc, prob, S_gpu, S_match, eps, U0, U_gpu, e_iso, label, **extra):
    """The end-to-end comparison against the oracle's update from S_match, its bounds and
    its record; asserts |dU| <= 1e-5 or within the measured-difference bound."""
    st, w, rho, eta = orc.weights(S_match, prob.lam)
    d = deltas(prob, eps, U0)
    delta = np.tensordot(w, d, axes=(0, 0))
    Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
    U_ref = U0.astype(np.float64) + Mx @ delta
    e2e = float(np.abs(U_gpu.astype(np.float64) - U_ref).max())
    bound, allowed = e2e_bounds(prob, S_match, S_gpu, d, w, delta, Mx)
    pred = first_order(prob, S_match, S_gpu, d, w, delta, Mx)
    resid = float(np.abs(U_gpu - U_ref - pred).max())
    fin = np.isfinite(S_match)
    rel = np.abs(S_gpu.astype(np.float64)[fin] - S_match[fin]) / np.maximum(np.abs(S_match[fin]), 1.0)
    record(check=label, K=prob.K, T=prob.T, lam=prob.lam, max_rel_dS=float(rel.max()) if rel.size else 0.0,
           dU_iso=e_iso, dU_e2e=e2e, dU_e2e_bound=bound + e_iso, dU_allowed_by_cost_bar=allowed + e_iso,
           dU_first_order=float(np.abs(pred).max()), first_order_residual=resid, **extra)
    print(f"{label} K={prob.K} T={prob.T}: max rel dS {rel.max() if rel.size else 0:.2e}, |dU| iso {e_iso:.2e} "
          f"e2e {e2e:.2e} (bound {bound + e_iso:.2e}, first-order {np.abs(pred).max():.2e}, residual {resid:.2e})",
          flush=True)
    assert e2e <= U_ATOL or e2e <= (bound + e_iso) * (1.0 + 1e-6) + 1e-12, \
        f"end-to-end |dU| {e2e:.3e} above U_ATOL and the bound {bound + e_iso:.3e}"
    return e2e, bound


def check_costs(orc, op, prob, cmap, params, x0, U0, eps, S, S_ref, impulses, near_cap):
    """The cost bar; returns S_match (oracle-side) and the per-sample bookkeeping."""
    fin = np.isfinite(S_ref)
    assert np.array_equal(np.isfinite(S), fin), "non-finite samples differ"
    events = _events(orc, op, prob, x0, U0, eps) if impulses else None
    S_match, near, flipped = match_costs(S, S_ref, events)
    err = np.where(fin, np.abs(np.where(fin, S.astype(np.float64), 0.0) - np.where(fin, S_match, 0.0))
                   / np.maximum(np.abs(np.where(fin, S_match, 0.0)), 1.0), 0.0)
    excluded = np.zeros(S.size, bool)
    if getattr(prob, "model", 0) == 1:
        excluded = branch_margins(orc, prob, cmap, params, x0, U0, eps) < NEAR_WINDOW
        assert excluded.mean() <= near_cap, f"{excluded.mean():.4f} of the samples pass the v_x branch point"
        err = np.where(excluded, 0.0, err)
    worst = int(np.argmax(err))
    assert err.max() <= COST_RTOL, \
        f"S_{worst}: gpu {S[worst]} oracle {S_match[worst]} (unmatched {S_ref[worst]}) rel {err.max():.3e}"
    info = dict(n_near_threshold=int(near.sum()), n_other_side=int(flipped.sum()),
                n_branch_excluded=int(excluded.sum()))
    return S_match, err, info


def check_results(orc, prob, cmap, params, x0, U0, S, Ug, it=0, impulses=False, near_cap=1e-3, label="IT",
                  **extra):
    """One iteration's GPU costs S and updated controls Ug (from U0, iteration it) against
    the oracle: the cost bar, the stage-isolated update (the oracle's weights and update
    on the GPU's S and the same noise) and the end-to-end comparison."""
    op = orc.OracleProblem(prob, cmap, params)
    eps = orc.noise(op, it)
    ref = orc.iterate(op, x0, U0, it)
    assert ref.status == orc.OK
    S_match, err, info = check_costs(orc, op, prob, cmap, params, x0, U0, eps, S, ref.S, impulses, near_cap)
    st2, w, rho, eta = orc.weights(S.astype(np.float64), prob.lam)
    delta = np.tensordot(w, deltas(prob, eps, U0), axes=(0, 0))
    Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
    U_iso = U0.astype(np.float64) + Mx @ delta
    e_iso = float(np.abs(Ug - U_iso).max())
    assert e_iso <= U_ATOL, f"stage-isolated |dU| {e_iso:.3e}"
    end_to_end(orc, prob, S, S_match, eps, U0, Ug, e_iso, label, it=it, **info, **extra)


def check_iteration(M, orc, prob, cmap, params, x0, U0, schedule, it=0, impulses=False, near_cap=1e-3):
    """One iteration against the oracle.  near_cap bounds the fraction of samples whose FP64
    trajectory passes the basis-function model's branch point (and are left out)."""
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
    S_match, err, info = check_costs(orc, op, prob, cmap, params, x0, U0, eps, S, ref.S, impulses, near_cap)
    # stage-isolated: oracle weights + update on the GPU's S and the same eps
    st2, w, rho, eta = orc.weights(S.astype(np.float64), prob.lam)
    delta = np.tensordot(w, deltas(prob, eps, U0), axes=(0, 0))
    Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
    U_iso = U0.astype(np.float64) + Mx @ delta
    e_iso = float(np.abs(Ug - U_iso).max())
    assert e_iso <= U_ATOL, f"stage-isolated |dU| {e_iso:.3e}"
    assert abs(rho_g - rho) <= 1e-6 * max(abs(rho), 1.0)
    np.testing.assert_allclose(delta_g, delta, rtol=0, atol=1e-6)
    end_to_end(orc, prob, S, S_match, eps, U0, Ug, e_iso, "IT", schedule=schedule, it=it, **info)
    return S, Ug


def check_cem(M, orc, prob, cmap, params, x0, U0, schedule, it=0, impulses=False, near_cap=1e-3):
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
    S_match, err, info = check_costs(orc, op, prob, cmap, params, x0, U0, eps, S, ref.S, impulses, near_cap)
    d = deltas(prob, eps, U0)
    Mx = orc.sgf_matrix(prob.T, prob.sg_window, prob.sg_order)
    # stage-isolated: the oracle's Algorithm 3 on the GPU's costs
    st2, w_iso, z_iso, n_iso = orc.weights_cem(S.astype(np.float64), zeta)
    delta_iso = np.tensordot(w_iso, d, axes=(0, 0))
    e_iso = np.abs(Ug - (U0.astype(np.float64) + Mx @ delta_iso)).max()
    assert e_iso <= U_ATOL, f"stage-isolated |dU| {e_iso:.3e}"
    np.testing.assert_allclose(delta_g, delta_iso, rtol=0, atol=1e-6)
    assert n_g == n_iso and z_g == np.float32(z_iso), (n_g, n_iso, z_g, z_iso)
    # end to end: the elite set from the oracle-side costs S_match may differ from the
    # GPU's only in samples within 1e-5 (relative) of the elite threshold, and U by that swap
    st3, w_ref, z_r, n_r = orc.weights_cem(S_match, zeta)
    U_ref = U0.astype(np.float64) + Mx @ np.tensordot(w_ref, d, axes=(0, 0))
    E_g, E_r = set(np.nonzero(w_iso)[0]), set(np.nonzero(w_ref)[0])
    swapped = sorted(E_g ^ E_r)
    for k in swapped:
        assert abs(S_match[k] - z_r) <= COST_RTOL * max(abs(z_r), 1.0), (k, S_match[k], z_r)
    pred = Mx @ ((d[sorted(E_g - E_r)].sum(axis=0) - d[sorted(E_r - E_g)].sum(axis=0)) / n_iso) if swapped else 0.0
    resid = float(np.abs(Ug - U_ref - pred).max())
    e2e = float(np.abs(Ug - U_ref).max())
    record(check="CEM", K=prob.K, T=prob.T, zeta=zeta, max_rel_dS=float(err.max()), dU_iso=float(e_iso),
           dU_e2e=e2e, swapped=len(swapped), swap_residual=resid, schedule=schedule, it=it, **info)
    print(f"CEM K={prob.K} T={prob.T} sched={schedule} zeta={zeta}: rel dS {err.max():.2e}, |dU| iso "
          f"{e_iso:.2e}, e2e {e2e:.2e}, swapped {len(swapped)}, e2e residual {resid:.2e}", flush=True)
    assert resid <= U_ATOL
    return S, Ug
