"""Benchmark: MPPI rollout steps/s (K x T per second) and iteration latency on one MI355X.

Workload: the paper-shaped configuration, K = 1920 samples, T = 100 steps, dt = 0.02,
the 6-32-32-4 tanh network (1412 parameters, Xavier-uniform, seed 0), a 2048 x 2048
elliptical track cost map at 0.05 m/cell, speed/slip/crash costs, lambda = 6.7,
Savitzky-Golay window 9.  One step = one MPPI iteration (noise, rollouts, weights,
weighted perturbation sum, smoothing, update) through the C ABI, warm-started from
the previous iteration's controls; all inputs are resident in HBM before timing.

Prints one JSON line with the throughput, the rollout kernel's roofline figures
(algorithmic FLOP of the dynamics network per launch over the kernel's average
duration, measured with HIP events on the library's stream) and the CPU oracle's
throughput on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector peak
NET_FLOP_PER_STEP = {32: 2 * (6 * 32 + 32 * 32 + 32 * 4), 64: 2 * (6 * 64 + 64 * 64 + 64 * 4)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--schedule", type=int, default=0, help="0 auto, 1 lane, 2 wave")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--latency-iters", type=int, default=200)
    return ap.parse_args()


def cpu_baseline(prob, cmap, params, x0, budget_s: float):
    """The CPU oracle (FP64, threads over samples) on full-size iterations of the same
    workload, repeated until about budget_s seconds have been spent."""
    import oracle
    nthreads = min(16, os.cpu_count() or 1)
    op = oracle.OracleProblem(prob, cmap, params, nthreads=nthreads)
    U = np.zeros((prob.T, 2), np.float32)
    t0 = time.perf_counter()
    n = 0
    while True:
        r = oracle.iterate(op, x0, U, n)
        U = r.U.astype(np.float32)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 1000:
            break
    return {"value": prob.K * prob.T * n / el, "unit": "steps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} full iterations (K={prob.K}, T={prob.T}), FP64, {nthreads} threads over samples, "
                      f"{el:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_1707_02342_amd import mppi as M

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    prob = synth.c2_problem(seed=0)
    cmap = synth.ellipse_map()
    params = synth.mlp_params(prob.hidden, 0)
    x0 = synth.C2_X0
    ctl = M.Controller(prob, cmap, params, stream=int(stream.cuda_stream), schedule=args.schedule)
    K, T = prob.K, prob.T

    for _ in range(args.warmup):
        ctl.iterate(x0)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # timed region: K iterations back to back, no per-launch events
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        ctl.iterate(x0)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1)
    ms_per_step = wall * 1e3 / args.steps
    value = K * T * args.steps / wall

    # the iteration kernel's average duration: HIP events around every launch on the
    # library's stream, over a second pass of the same length (the events themselves
    # add stream markers, so this pass is not the throughput one)
    M.mppi_set_timing(ctl.ctx, True)
    for _ in range(args.steps):
        ctl.iterate(x0)
    (t_roll, _), (n_roll, _) = M.mppi_get_timing(ctl.ctx)
    M.mppi_set_timing(ctl.ctx, False)

    # host-observed latency: iterate + copy of U back to the host, one at a time
    lat = []
    for _ in range(args.latency_iters):
        t1 = time.perf_counter()
        ctl.iterate(x0)
        ctl.controls()
        lat.append((time.perf_counter() - t1) * 1e6)
    lat = np.array(lat)

    roll_ms = t_roll / max(n_roll, 1)
    flop = NET_FLOP_PER_STEP[prob.hidden] * K * T
    achieved = flop / (roll_ms * 1e-3) / 1e12
    out = {
        "metric": "MPPI rollout steps/sec (K×T per s) and iteration latency at K=1920,T=100",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper-shaped MPPI iteration: K=1920, T=100, 6-32-32-4 tanh network, "
                               "2048x2048 elliptical track map, SGF window 9",
                   "K": K, "T": T, "hidden": prob.hidden, "schedule": ctl.schedule},
        "latency_us": {"device_per_iteration": dev_ms * 1e3 / args.steps,
                       "rollout_kernel": roll_ms * 1e3,
                       "host_p50": float(np.percentile(lat, 50)), "host_p99": float(np.percentile(lat, 99))},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "rollout", "flop_per_launch": flop},
    }
    ctl.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, cmap, params, x0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
