"""Closed-loop lap evaluation on a synthetic plant, in the manner of the paper's track
experiments (Section VII, Table 3): the controller drives the plant around the
elliptical track for a number of laps, each lap is classified as a success or a
failure, the first lap is discarded (it starts from rest-like conditions), and the
success rate, the lap time (mean and standard deviation over successful laps) and the
speed range are reported.

Every control step runs in the library (`mppi_run_receding`: iteration, shift and the
plant step in one launch); this module only segments the executed trajectory into
laps.  A lap fails when the vehicle leaves the track anywhere in it (the cost map
exceeds the crash threshold at an executed state, looked up with the kernels' own
interpolation through `mppi_costmap_values`) or the state stops being finite.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import mppi as M


@dataclass
class Track:
    """An elliptical centre line: centre (c_x, c_y) and semi-axes (a, b)."""
    center: tuple = (51.2, 51.2)
    semi_axes: tuple = (40.0, 25.0)


def lap_progress(X: np.ndarray, track: Track, direction: int = 1) -> np.ndarray:
    """Progress along the track in laps, from the first state: the unwrapped angle of the
    position in the ellipse's own coordinates divided by 2 pi, counted positive in the
    driving direction (+1 counter-clockwise, -1 clockwise)."""
    cx, cy = track.center
    a, b = track.semi_axes
    ang = np.unwrap(np.arctan2((X[:, 1] - cy) / b, (X[:, 0] - cx) / a))
    return direction * (ang - ang[0]) / (2.0 * np.pi)


def crossing_times(progress: np.ndarray, dt: float) -> np.ndarray:
    """Times (seconds, linearly interpolated between steps) at which the progress first
    reaches 1, 2, 3, ... laps."""
    out = []
    k = 1
    for i in range(1, len(progress)):
        while progress[i] >= k and progress[i - 1] < k:
            f = (k - progress[i - 1]) / (progress[i] - progress[i - 1])
            out.append((i - 1 + f) * dt)
            k += 1
    return np.array(out)


def lap_metrics(X: np.ndarray, h: np.ndarray, dt: float, track: Track, direction: int,
                crash_threshold: float, discard_first: bool = True) -> dict:
    """Lap statistics of one run: X the executed states [n][7], h the cost map at each
    state's position [n]."""
    prog = lap_progress(X, track, direction)
    tc = crossing_times(prog, dt)
    bounds = np.concatenate([[0.0], tc])                  # lap k runs from bounds[k] to bounds[k + 1]
    laps = []
    for k in range(len(tc)):
        i0 = int(np.floor(bounds[k] / dt))
        i1 = min(int(np.ceil(bounds[k + 1] / dt)), len(X) - 1)
        seg = slice(i0, i1 + 1)
        ok = bool(np.all(np.isfinite(X[seg])) and np.all(h[seg] <= crash_threshold))
        laps.append({"time": float(bounds[k + 1] - bounds[k]), "success": ok,
                     "v_min": float(np.min(X[seg, 4])), "v_max": float(np.max(X[seg, 4]))})
    counted = laps[1:] if discard_first else laps
    good = [l for l in counted if l["success"]]
    times = np.array([l["time"] for l in good])
    return {
        "laps": len(counted),
        "success_pct": 100.0 * len(good) / len(counted) if counted else None,
        "lap_time_mean": float(times.mean()) if len(good) else None,
        "lap_time_std": float(times.std()) if len(good) else None,
        "speed_min": min(l["v_min"] for l in good) if good else None,
        "speed_max": max(l["v_max"] for l in good) if good else None,
        "per_lap": laps,
    }


def drive(ctl, x0, n_laps: int, dt: float, track: Track, direction: int = 1,
          max_steps: int = 200_000, block: int = 1000):
    """Runs the receding-horizon loop from x0 until n_laps laps are complete (or
    max_steps); returns the executed states [n + 1][7] and controls [n][2]."""
    x = np.asarray(x0, np.float32).copy()
    xs, us = [x[None]], []
    steps = 0
    while steps < max_steps:
        n = min(block, max_steps - steps)
        uh, xh, _ = M.mppi_run_receding(ctl.ctx, x, n)
        xs.append(xh[1:])
        us.append(uh)
        x = xh[-1]
        steps += n
        X = np.concatenate(xs)
        if not np.all(np.isfinite(x)):
            break
        if lap_progress(X, track, direction)[-1] >= n_laps:
            break
    return np.concatenate(xs), np.concatenate(us) if us else np.zeros((0, 2), np.float32)


def evaluate(ctl, x0, n_laps: int, dt: float, track: Track, direction: int, crash_threshold: float,
             max_steps: int = 200_000) -> dict:
    """drive() then lap_metrics() with the cost map looked up on the GPU."""
    X, U = drive(ctl, x0, n_laps, dt, track, direction, max_steps)
    fin = np.all(np.isfinite(X), axis=1)
    h = np.full(len(X), np.inf, np.float32)
    if fin.any():
        h[fin] = M.mppi_costmap_values(ctl.ctx, X[fin, :2])
    out = lap_metrics(X, h, dt, track, direction, crash_threshold)
    out["steps"] = len(U)
    return out
