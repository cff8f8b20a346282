"""Benchmark: MPPI rollout steps/s (K x T per second) and iteration latency on one MI355X.

Workload: the paper-shaped receding-horizon configuration, K = 1920 samples, T = 100
steps, dt = 0.02, the 6-32-32-4 tanh network (1412 parameters, Xavier-uniform, seed 0),
a 2048 x 2048 elliptical track cost map at 0.05 m/cell, speed/slip/crash costs,
lambda = 6.7, Savitzky-Golay window 9; 100 warm-started iterations per Philox seed
0..9 on a synthetic plant (the same network, noise-free).  One step = one control
step: an MPPI iteration (noise, rollouts, weights, weighted perturbation sum,
smoothing, update), the shift of U and the plant step.  The timed region drives each
seed's 100-step block through the C ABI as one mppi_run_receding_device call on a
device-resident plant state (one multi-step launch on this workload); all inputs are
resident in HBM before timing, and the timed region allocates nothing and copies
nothing to the host.

Prints one JSON line with the throughput, the device time per step inside the
launches, the single-step launch figures (mppi_step_device: back to back and per
launch), host latencies (eager and HIP-graph-replayed), the roofline figures
(algorithmic FLOP of the dynamics network over the device time per step, measured with
HIP events on the library's stream), the precision / batched / differentiation forms,
and the CPU oracle's throughput on a bounded sample of the same workload.
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

PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector (and FP32 matrix) peak
PEAK_BF16_TFLOPS = 2500.0         # MI355X published dense BF16/FP16 matrix peak
VALU_LANE_SLOTS_PER_S = 256 * 64 * 2.4e9   # CUs x lanes x clock: one FP32 op per lane per cycle
TRAFFIC_FILE = ROOT / "profiles" / "rollout_wave_split_k1920_t100_traffic.json"
TRAFFIC_KERNEL = "rollout_wave_split_kernel<0, true>"   # the multi-step launch of the timed region
STEPS_PER_LAUNCH = 100                                 # receding steps per launch in the timed region
# the sources the benchmarked kernel (rollout_wave_kernel<32, 4, 0>) is built from: stored
# counter readings are used only while these files are unchanged
KERNEL_SOURCES = ["kernels_wave_split.hip", "kernels_wave.hip", "wave_common.hip.h", "kernels_common.hip.h", "device_common.h",
                  "mppi_types.h"]
NET_FLOP_PER_STEP = {32: 2 * (6 * 32 + 32 * 32 + 32 * 4), 64: 2 * (6 * 64 + 64 * 64 + 64 * 4)}
# basis-function model: Theta^T phi (25 x 4 multiply-adds) plus about 40 operations forming phi
BASIS_FLOP_PER_STEP = 2 * 25 * 4 + 40
# adjoint rollout per sample and step (h = 32): the forward network recomputed from the
# checkpoint (2688) and the reverse sweep -- per layer the transposed product for the
# input cotangent and the outer product for the weight gradient, each the size of the
# forward product (2 x 2688)
ADJOINT_FLOP_PER_STEP = 3 * NET_FLOP_PER_STEP[32]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="receding-horizon steps (100 per seed in turn)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--schedule", type=int, default=0, help="0 auto, 1 lane, 2 wave")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--latency-iters", type=int, default=300)
    ap.add_argument("--no-forms", action="store_true", help="skip the precision/batched/differentiation forms")
    ap.add_argument("--precision-only", action="store_true",
                    help="only time the precision form (K=16384 and 65536), print its JSON and exit")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched form (512 instances; for profiling its kernel)")
    ap.add_argument("--differentiation-only", action="store_true",
                    help="only time the differentiation form (K=4096, T=100), print its JSON and exit")
    ap.add_argument("--write-traffic", metavar="PMC_DIR",
                    help="reduce rocprofv3 FETCH_SIZE/WRITE_SIZE runs under PMC_DIR to the stored traffic "
                         "record under profiles/ and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 256 MiB device-to-device copy five times (reference for the "
                         "profiler's HBM byte counters) and exit")
    return ap.parse_args()


COPY_BYTES = 256 << 20


def calibrate_copy():
    """Five copies of COPY_BYTES between two device buffers: a kernel whose HBM traffic
    is known (COPY_BYTES read and COPY_BYTES written per launch), against which the
    FETCH_SIZE and WRITE_SIZE counters are scaled."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": COPY_BYTES, "launches": 5}), flush=True)


# the sources of the precision form's kernel (rollout_quad_kernel): stored error records
# are shown beside the measured speedups only while these files are unchanged
QUAD_SOURCES = ["kernels_quad.hip", "kernels_common.hip.h", "device_common.h", "mppi_types.h"]
PARITY_RECORDS = ROOT / "profiles" / "precision_errors.jsonl"


def kernel_sources_sha256(names=None) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in (KERNEL_SOURCES if names is None else names):
        h.update((ROOT / "paper_1707_02342_amd" / "csrc" / name).read_bytes())
    return h.hexdigest()


def precision_errors(K: int):
    """The precision form's error against the FP64 oracle per seed (max relative S error
    and max |dU|, total and with the weights rounded to the operand type), from the
    records the GPU parity tests write (tests/test_gpu_forms.py, kept under profiles/),
    or None when the quad kernel's sources changed after they were taken."""
    if not PARITY_RECORDS.exists():
        return None
    sha = kernel_sources_sha256(QUAD_SOURCES)
    out = {}
    for line in PARITY_RECORDS.read_text().splitlines():
        r = json.loads(line)
        if r.get("check") != "precision" or r.get("K") != K or r.get("schedule") != 4:
            continue
        if r.get("sources_sha256") != sha:
            continue
        name = {1: "bf16", 2: "fp16"}[r["precision"]]
        out.setdefault(name, {})[str(r["seed"])] = {k: r[k] for k in (
            "S_rel_max", "S_rel_max_rounded_weights", "dU_max", "dU_max_rounded_weights")}
    return out or None


def stored_traffic():
    """HBM bytes per receding step of the benchmarked kernel (a launch's bytes over its
    steps) from the profiler's FETCH_SIZE and WRITE_SIZE counters (scaled by a copy of
    known size), or None when the kernel's sources changed after the counters were
    taken."""
    if not TRAFFIC_FILE.exists():
        return None
    rec = json.loads(TRAFFIC_FILE.read_text())
    if rec.get("sources_sha256") != kernel_sources_sha256():
        return None
    return rec["traffic_bytes_per_step"]


def write_traffic(pmc_dir: str):
    """Reduce four rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE of the benchmark and
    of --calibrate-copy, CSV output under pmc_dir/{FETCH_SIZE,WRITE_SIZE,FETCH_SIZE_copy,
    WRITE_SIZE_copy}/) to the HBM bytes per receding step of the multi-step rollout
    kernel (the median over its 100-step launches, divided by 100)."""
    import csv
    import glob

    def per_dispatch(sub, match):
        f = glob.glob(os.path.join(pmc_dir, sub, "*_counter_collection.csv"))[0]
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(f)) if match(r["Kernel_Name"])]
        return float(np.median(vals)), len(vals)

    is_roll = lambda n: TRAFFIC_KERNEL in n
    is_copy = lambda n: "copyBuffer" in n or "elementwise" in n
    fetch, nf = per_dispatch("FETCH_SIZE", is_roll)
    write, nw = per_dispatch("WRITE_SIZE", is_roll)
    # the copy kernel's dispatches: the largest reading is the 256 MiB copy
    def largest(sub):
        f = glob.glob(os.path.join(pmc_dir, sub, "*_counter_collection.csv"))[0]
        return max(float(r["Counter_Value"]) for r in csv.DictReader(open(f)) if is_copy(r["Kernel_Name"]))
    kib = COPY_BYTES / 1024.0
    fetch_scale = kib / largest("FETCH_SIZE_copy")
    write_scale = kib / largest("WRITE_SIZE_copy")
    per_launch = (fetch * fetch_scale + write * write_scale) * 1024.0
    rec = {"kernel": TRAFFIC_KERNEL,
           "workload": "K=1920, T=100, 6-32-32-4 network, 2048x2048 map (bench.py default), "
                       f"{STEPS_PER_LAUNCH} receding steps per launch",
           "sources_sha256": kernel_sources_sha256(),
           "fetch_size_kib_per_launch_median": fetch, "fetch_dispatches": nf, "fetch_scale": fetch_scale,
           "write_size_kib_per_launch_median": write, "write_dispatches": nw, "write_scale": write_scale,
           "traffic_bytes_per_launch": per_launch, "steps_per_launch": STEPS_PER_LAUNCH,
           "traffic_bytes_per_step": per_launch / STEPS_PER_LAUNCH,
           "commands": ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/FETCH_SIZE -o c2 -- "
                        "python3 bench.py --steps 100 --warmup 5 --no-cpu --no-forms --latency-iters 5",
                        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/WRITE_SIZE -o c2 -- "
                        "python3 bench.py --steps 100 --warmup 5 --no-cpu --no-forms --latency-iters 5",
                        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/FETCH_SIZE_copy -o copy -- "
                        "python3 bench.py --calibrate-copy",
                        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/WRITE_SIZE_copy -o copy -- "
                        "python3 bench.py --calibrate-copy",
                        "python3 bench.py --write-traffic <dir>"]}
    TRAFFIC_FILE.parent.mkdir(exist_ok=True)
    TRAFFIC_FILE.write_text(json.dumps(rec, indent=1) + "\n")
    print(json.dumps(rec), flush=True)


def host_cpu():
    """The host's CPU model (from /proc/cpuinfo) and the cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count() or 1
    return model, visible


def cpu_baseline(prob, cmap, params, x0, budget_s: float):
    """The CPU oracle (FP64, threads over samples) on full-size iterations of the same
    workload, repeated until about budget_s seconds have been spent.  Threads: the
    process's CPU share (OMP_NUM_THREADS when set -- 16 per GPU on the GPU hosts --
    capped by the cores it may run on)."""
    import oracle
    model, visible = host_cpu()
    share = int(os.environ.get("OMP_NUM_THREADS", visible) or visible)
    nthreads = max(1, min(share, visible))
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
            "cpu_model": model, "host_cores_visible": visible,
            "sample": f"{n} full iterations (K={prob.K}, T={prob.T}), FP64, {nthreads} threads over samples, "
                      f"{el:.1f} s, on {model}"}


def _timed_iterations(ctl, x0, n, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(n):
        ctl.iterate(x0)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n          # ms per iteration


def measure_precision(M, stream, iters: int = 30):
    """The precision form: K=16384 (top level; one wave of 16 samples per SIMD) and
    K=65536 ("k65536"; four per SIMD), T=100, 6-64-64-4 network, FP32 and BF16 / FP16
    matrix-core operands with FP32 accumulation."""
    import synth
    params = synth.mlp_params(64, 0)
    cmap = synth.ring_map()
    flop = NET_FLOP_PER_STEP[64]
    # rooflines: FP32 on the matrix cores against the FP32 matrix peak; BF16/FP16 are
    # bound by the vector ALU (tanh: exp and rcp at quarter rate + 3 FMA = 11 slots, 128
    # per step at h = 64, plus ~150 other slots) -- reported against that bound and,
    # for reference, as a fraction of the BF16/FP16 matrix peak
    valu_steps_peak = VALU_LANE_SLOTS_PER_S / (128 * 11 + 150)

    def precision_at(K):
        prob = synth.c3_problem(K=K, seed=0)
        prec = {}
        for name, p in (("fp32", M.MPPI_PREC_FP32), ("bf16", M.MPPI_PREC_BF16), ("fp16", M.MPPI_PREC_FP16)):
            ctl = M.Controller(prob, cmap, params, stream=int(stream.cuda_stream), precision=p)
            for _ in range(3):
                ctl.iterate(synth.C1_X0)
            ms = _timed_iterations(ctl, synth.C1_X0, iters, stream)
            ctl.close()
            prec[name] = {"ms_per_iteration": ms, "steps_per_s": prob.K * prob.T / (ms * 1e-3)}
        f32_tflops = prec["fp32"]["steps_per_s"] * flop / 1e12
        prec["fp32"]["roofline"] = {"bound": "mfma", "achieved": f32_tflops, "peak": PEAK_FP32_TFLOPS,
                                    "unit": "TFLOP/s", "frac": f32_tflops / PEAK_FP32_TFLOPS}
        for name in ("bf16", "fp16"):
            st = prec[name]["steps_per_s"]
            prec[name]["roofline"] = {"bound": "alu", "achieved": st / 1e9, "peak": valu_steps_peak / 1e9,
                                      "unit": "Gsteps/s", "frac": st / valu_steps_peak,
                                      "mfma_frac": st * flop / 1e12 / PEAK_BF16_TFLOPS}
        prec["bf16_speedup_vs_fp32"] = prec["fp32"]["ms_per_iteration"] / prec["bf16"]["ms_per_iteration"]
        prec["fp16_speedup_vs_fp32"] = prec["fp32"]["ms_per_iteration"] / prec["fp16"]["ms_per_iteration"]
        prec["workload"] = f"K={K}, T=100, 6-64-64-4 network, 256x256 ring map"
        prec["error_vs_fp64_per_seed"] = precision_errors(K)
        return prec

    prec = precision_at(16384)
    prec["k65536"] = precision_at(65536)
    return prec


def measure_differentiation(M, stream, iters: int = 30):
    """The differentiation form: K=4096, T=100, the free-energy objective plus its adjoint
    gradient with checkpoints every 10 steps; wall time per value-and-gradient, and the
    adjoint rollout kernel's duration and roofline (HIP events on the library's stream)."""
    import synth
    prob = synth.c5_problem(seed=0)
    U = synth.random_controls(prob.T, 0, scale=0.2)
    with M.Controller(prob, synth.ring_map(), synth.mlp_params(32, 0), stream=int(stream.cuda_stream)) as c:
        c.set_controls(U)
        for _ in range(2):
            c.objective(synth.C1_X0, 0, 10)
            c.objective_backward()
        t0 = time.perf_counter()
        for _ in range(iters):
            c.objective(synth.C1_X0, 0, 10)
            c.objective_backward()
        ms = (time.perf_counter() - t0) * 1e3 / iters
        # kernel durations (HIP events on the library's stream): the objective's forward
        # launch (slot 0) and the adjoint rollout kernel (slot 1)
        M.mppi_set_timing(c.ctx, True)
        for _ in range(iters):
            c.objective(synth.C1_X0, 0, 10)
            c.objective_backward()
        (f_ms, a_ms), (f_n, a_n) = M.mppi_get_timing(c.ctx)
        M.mppi_set_timing(c.ctx, False)
    adj_ms = a_ms / a_n
    adj_tf = ADJOINT_FLOP_PER_STEP * prob.K * prob.T / (adj_ms * 1e-3) / 1e12
    return {"ms_per_value_and_gradient": ms,
            "forward_kernel_ms": f_ms / f_n, "adjoint_kernel_ms": adj_ms,
            "roofline": {"bound": "alu", "achieved": adj_tf, "peak": PEAK_FP32_TFLOPS,
                         "unit": "TFLOP/s", "frac": adj_tf / PEAK_FP32_TFLOPS,
                         "kernel": "adjoint_wave_kernel",
                         "flop_per_launch": ADJOINT_FLOP_PER_STEP * prob.K * prob.T},
            "workload": "K=4096, T=100, checkpoints every 10 steps, 1612 gradient entries"}


def measure_batched(M, iters: int = 30):
    """The batched form: 512 instances (K_i in 512..4096, T_i in 50..150) advanced by one
    replayed graph launch per iteration (the first iterate autotunes and captures it)."""
    import synth
    inst = synth.c4_instances(512, seed=0)
    Ks, Ts = [b.K for b in inst], [b.T for b in inst]
    x0s = np.stack([b.x0 for b in inst])
    with M.Batch(synth.c2_problem(seed=0), Ks, Ts, synth.ellipse_map(), synth.mlp_params(32, 0)) as b:
        b.iterate(x0s)              # autotunes and captures the launch
        b.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            b.iterate(x0s)
        b.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / iters
        grid, order, tuned_us, tiles = b.schedule()
    work = float(sum(k * t for k, t in zip(Ks, Ts)))
    bt = work * NET_FLOP_PER_STEP[32] / (ms * 1e-3) / 1e12
    return {"ms_per_iteration": ms, "steps_per_s": work / (ms * 1e-3), "instances": len(Ks),
            "roofline": {"bound": "mfma", "achieved": bt, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": bt / PEAK_FP32_TFLOPS},
            "grid": grid, "order": order,
            "tiles": {1: "lane schedule, 256 samples per tile",
                      4: "quad schedule, 64 samples per tile"}.get(tiles, tiles),
            "workload": "512 instances, K_i in {512..4096}, T_i in {50..150}, 2048x2048 map"}


def measure_forms(M, stream, iters: int = 30, laps_per_setting: int = 3):
    """The three added forms on their own workloads (synthetic, seeded):
    precision: K=16384 and K=65536, T=100, 6-64-64-4 network, one iteration in FP32 and
      with BF16 / FP16 matrix-core operands (FP32 accumulation);
    batched: 512 instances (K_i in 512..4096, T_i in 50..150) advanced by one replayed
      graph launch per iteration;
    differentiation: K=4096, T=100, free-energy objective plus its adjoint gradient
      with checkpoints every 10 steps;
    exploration: the paper-shaped receding-horizon step with the parameter table's
      lambda, gamma and Sigma and 1 % of the samples drawn around zero;
    cem: the same step with Algorithm 3's weights (the best 20 % averaged);
    basis: the paper-shaped step with the basis-function model;
    laps: closed-loop lap statistics (measure_laps)."""
    import torch
    import synth
    out = {"precision": measure_precision(M, stream, iters)}

    out["batched"] = measure_batched(M, iters)

    out["differentiation"] = measure_differentiation(M, stream, iters)

    emap = synth.ellipse_map()
    for name, prob, desc in (
            ("exploration", synth.explore_problem(seed=0),
             "K=1920 (19 exploration samples), T=100, lambda=12.5, gamma=0.1, Sigma=Diag(0.0306, 0.0506), "
             "receding horizon, 2048x2048 map"),
            ("cem", synth.cem_problem(seed=0),
             "Algorithm 3 weights (384 elite of K=1920), T=100, gamma=0.1, Sigma=Diag(0.0306, 0.0506), "
             "receding horizon, 2048x2048 map"),
            ("basis", synth.basis_problem(seed=0),
             "basis-function model (25 bases, synthetic Theta) in place of the network, K=1920, T=100, "
             "receding horizon, 2048x2048 map")):
        params = synth.basis_theta(0) if prob.model == 1 else synth.mlp_params(32, 0)
        with M.Controller(prob, emap, params, stream=int(stream.cuda_stream)) as c:
            M.mppi_run_receding(c.ctx, synth.C2_X0, 20)
            torch.cuda.synchronize()
            n_blk = 3
            t0 = time.perf_counter()
            for _ in range(n_blk):
                M.mppi_run_receding(c.ctx, synth.C2_X0, 100)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / (100 * n_blk)
            sched = c.schedule
            M.mppi_set_timing(c.ctx, True)
            M.mppi_run_receding(c.ctx, synth.C2_X0, 100)
            launch = M.mppi_get_timing_samples(c.ctx)
            M.mppi_set_timing(c.ctx, False)
        st = prob.K * prob.T / (ms * 1e-3)
        launch_ms = float(np.mean(launch))
        flop = BASIS_FLOP_PER_STEP if prob.model == 1 else NET_FLOP_PER_STEP[32]
        tf = flop * prob.K * prob.T / (launch_ms * 1e-3) / 1e12
        out[name] = {"ms_per_step": ms, "steps_per_s": st, "schedule": sched,
                     "launch_us": {"mean": launch_ms * 1e3, "p50": float(np.percentile(launch, 50)) * 1e3,
                                   "p99": float(np.percentile(launch, 99)) * 1e3},
                     "roofline": {"bound": "alu", "achieved": tf, "peak": PEAK_FP32_TFLOPS,
                                  "unit": "TFLOP/s", "frac": tf / PEAK_FP32_TFLOPS},
                     "workload": desc}
    out["laps"] = measure_laps(M, emap, n_counted=laps_per_setting)
    return out


def measure_laps(M, emap, n_counted: int = 3):
    """Table 3 in the synthetic setting: the IT and CEM controllers (parameter table,
    basis-function model as both the controller's model and the plant) at speed targets
    6, 8.5 and 11 m/s, counter-clockwise (CC) and clockwise (C), n_counted laps each
    after a discarded first lap."""
    import synth
    from paper_1707_02342_amd import laps
    rows = []
    t0 = time.perf_counter()
    steps = 0
    for weighting, wname in ((0, "IT-MPC-BF"), (1, "CEM-BF")):
        for v_des in (6.0, 8.5, 11.0):
            for direction, dname in ((1, "CC"), (-1, "C")):
                cost = synth.c2_cost()
                cost.v_des = v_des
                prob = synth.with_(synth.explore_problem(0), model=1, weighting=weighting, elite=0.8, cost=cost)
                x0 = synth.ellipse_pose(0.0, 4.0)
                if direction < 0:
                    x0[2] += np.pi
                with M.Controller(prob, emap, synth.basis_theta(0)) as c:
                    m = laps.evaluate(c, x0, n_counted + 1, prob.dt, laps.Track(), direction,
                                      prob.cost.map_thresh, max_steps=60_000)
                steps += m["steps"]
                rows.append({"setting": f"{wname} {v_des:g} m/s {dname}", "laps": m["laps"],
                             "success_pct": m["success_pct"], "lap_time_s": m["lap_time_mean"],
                             "lap_time_std_s": m["lap_time_std"], "speed_min": m["speed_min"],
                             "speed_max": m["speed_max"]})
    wall = time.perf_counter() - t0
    return {"rows": rows, "control_steps": steps, "wall_s": wall,
            "workload": "synthetic plant = the basis-function model, 2048x2048 elliptical track, K=1920, T=100, "
                        "parameter table (lambda 12.5, gamma 0.1, Sigma Diag(0.0306, 0.0506), 1 % exploration)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.write_traffic:
        write_traffic(args.write_traffic)
        return
    import torch
    import synth
    from paper_1707_02342_amd import mppi as M

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.precision_only:
        print(json.dumps({"precision": measure_precision(M, stream, iters=10)}), flush=True)
        return
    if args.differentiation_only:
        print(json.dumps({"differentiation": measure_differentiation(M, stream, iters=10)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": measure_batched(M, iters=30)}), flush=True)
        return
    cmap = synth.ellipse_map()
    prob = synth.c2_problem(seed=0)
    params = synth.mlp_params(prob.hidden, 0)
    x0 = synth.C2_X0
    K, T = prob.K, prob.T
    sid = int(stream.cuda_stream)
    # one controller per Philox seed 0..9 (U = 0, iteration 0); each timed block of up
    # to 100 steps is a warm-started receding-horizon run of one seed from x0
    ctls = [M.Controller(synth.c2_problem(seed=s), cmap, params, stream=sid, schedule=args.schedule)
            for s in range(10)]
    schedule = ctls[0].schedule
    # each controller's plant state lives on the device; a control step is
    # mppi_step_device (iteration, shift and plant step in one launch, no host copy)
    xdev = [torch.tensor(x0, device="cuda") for _ in ctls]
    x0_t = torch.from_numpy(x0.copy())

    def reset_all():
        for c, xd in zip(ctls, xdev):
            c.set_controls(np.zeros((T, 2), np.float32))
            c.iteration = 0
            xd.copy_(x0_t)
        torch.cuda.synchronize()

    def receding(n_steps, single=False):
        """n_steps control steps: blocks of up to 100 warm-started steps, one Philox seed
        per block in turn, all enqueued back to back.  A block is one
        mppi_run_receding_device call (one multi-step launch on this workload), or with
        single=True one mppi_step_device launch per step."""
        done, blk = 0, 0
        while done < n_steps:
            n = min(STEPS_PER_LAUNCH, n_steps - done)
            ctx, ptr = ctls[blk % 10].ctx, xdev[blk % 10].data_ptr()
            if single:
                for _ in range(n):
                    M.mppi_step_device(ctx, ptr)
            else:
                M.mppi_run_receding_device(ctx, ptr, n)
            done += n
            blk += 1

    # per-launch device time: HIP events around every launch on the library's stream,
    # over the same steps from the same start (the events add stream markers, so this
    # pass is not the throughput one).  These passes run before the timed region, so that
    # it starts on a device already at its steady clocks and caches.
    reset_all()
    n_timed = max(args.steps, 500)
    receding(n_timed)                                # untimed: every controller's first launches
    torch.cuda.synchronize()
    reset_all()
    for c in ctls:
        M.mppi_set_timing(c.ctx, True)
    receding(n_timed)
    blocks = np.concatenate([M.mppi_get_timing_samples(c.ctx) for c in ctls])
    for c in ctls:
        M.mppi_set_timing(c.ctx, False)
    t_roll = float(blocks.sum()) / n_timed          # device ms per control step inside the launches
    # one launch per step (mppi_step_device), for the per-launch latency figures
    reset_all()
    for c in ctls:
        M.mppi_set_timing(c.ctx, True)
    receding(n_timed, single=True)
    samples = np.concatenate([M.mppi_get_timing_samples(c.ctx) for c in ctls])
    for c in ctls:
        M.mppi_set_timing(c.ctx, False)
    torch.cuda.synchronize()
    reset_all()
    t0s = time.perf_counter()
    receding(n_timed, single=True)
    torch.cuda.synchronize()
    single_step_us = (time.perf_counter() - t0s) * 1e6 / n_timed

    # host-observed latency of a control step, state in -> u_0 on the host: eager
    # (mppi_iterate + mppi_shift) and as a replayed HIP graph of mppi_step_device
    c = ctls[0]
    reset_all()
    lat_eager = []
    x = x0.copy()
    for _ in range(args.latency_iters):
        t1 = time.perf_counter()
        c.iterate(x)
        u0 = c.shift()
        lat_eager.append((time.perf_counter() - t1) * 1e6)
        x = c.plant_step(x, u0)
    reset_all()
    gs = torch.cuda.Stream()
    with M.Controller(prob, cmap, params, stream=int(gs.cuda_stream), schedule=args.schedule) as cg:
        xd = torch.tensor(x0, device="cuda")
        ud = torch.zeros(2, device="cuda")
        with torch.cuda.stream(gs):
            M.mppi_step_device(cg.ctx, xd.data_ptr(), ud.data_ptr())
        gs.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=gs):
            M.mppi_step_device(cg.ctx, xd.data_ptr(), ud.data_ptr())
        lat_graph = []
        for _ in range(args.latency_iters):
            t1 = time.perf_counter()
            g.replay()
            ud.cpu()
            lat_graph.append((time.perf_counter() - t1) * 1e6)
        del g
    lat_eager, lat_graph = np.array(lat_eager), np.array(lat_graph)

    # warm-up: `warmup` untimed control steps (one multi-step call), then all restart
    # from x0, U = 0, iteration 0
    reset_all()
    if args.warmup:
        M.mppi_run_receding_device(ctls[0].ctx, xdev[0].data_ptr(), args.warmup)
    torch.cuda.synchronize()
    reset_all()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # timed region: `steps` receding-horizon control steps (iteration, shift and plant
    # step), no per-launch events, no allocation, no host copy
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    receding(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1)
    ms_per_step = wall * 1e3 / args.steps
    value = K * T * args.steps / wall

    roll_ms = t_roll
    flop = NET_FLOP_PER_STEP[prob.hidden] * K * T
    achieved = flop / (roll_ms * 1e-3) / 1e12
    traffic = stored_traffic() if schedule == M.MPPI_SCHED_WAVE else None
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
        "config": {"workload": "paper-shaped receding-horizon MPPI: K=1920, T=100, 6-32-32-4 tanh network, "
                               "2048x2048 elliptical track map, SGF window 9, 100 warm-started iterations "
                               "per Philox seed 0-9 on a synthetic plant; one step = iteration + shift + "
                               "plant step",
                   "K": K, "T": T, "hidden": prob.hidden, "schedule": schedule,
                   "launch": "mppi_run_receding_device, one launch per 100-step block"},
        "latency_us": {"step_device_back_to_back": dev_ms * 1e3 / args.steps,
                       "kernel_per_step": roll_ms * 1e3,
                       "single_step_launches_back_to_back": single_step_us,
                       "single_step_launch_mean": float(np.mean(samples)) * 1e3,
                       "single_step_launch_p50": float(np.percentile(samples, 50)) * 1e3,
                       "single_step_launch_p99": float(np.percentile(samples, 99)) * 1e3,
                       "host_eager_p50": float(np.percentile(lat_eager, 50)),
                       "host_eager_p99": float(np.percentile(lat_eager, 99)),
                       "host_graph_p50": float(np.percentile(lat_graph, 50)),
                       "host_graph_p99": float(np.percentile(lat_graph, 99))},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "kernel": "rollout_wave_split_kernel<kModelNet, true>, per receding step of its "
                               f"{STEPS_PER_LAUNCH}-step launches", "flop_per_step": flop},
    }
    for cc in ctls:
        cc.close()
    if not args.no_forms:
        out["forms"] = measure_forms(M, stream)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, cmap, params, x0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
