"""Host logic of the closed-loop lap harness (paper_1707_02342_amd.laps): lap
segmentation, interpolated lap times and lap classification against trajectories
with closed-form answers."""
import math

import numpy as np

from paper_1707_02342_amd import laps

TRACK = laps.Track()


def _ellipse_traj(phi0, omega, dt, n, direction=1, v=5.0):
    t = np.arange(n) * dt
    phi = phi0 + direction * omega * t
    (cx, cy), (a, b) = TRACK.center, TRACK.semi_axes
    X = np.zeros((n, 7))
    X[:, 0] = cx + a * np.cos(phi)
    X[:, 1] = cy + b * np.sin(phi)
    X[:, 4] = v + 0.1 * np.sin(3 * t)
    return X


def test_lap_times_of_constant_angular_rate():
    # phi advances at omega rad/s: every lap takes exactly 2 pi / omega seconds
    dt, omega = 0.02, 0.17
    for direction in (1, -1):
        X = _ellipse_traj(0.3, omega, dt, 20000, direction)
        tc = laps.crossing_times(laps.lap_progress(X, TRACK, direction), dt)
        assert len(tc) == math.floor(omega * dt * 19999 / (2 * math.pi))
        np.testing.assert_allclose(np.diff(np.concatenate([[0.0], tc])), 2 * math.pi / omega, rtol=1e-6)


def test_wrong_direction_counts_no_laps():
    X = _ellipse_traj(0.0, 0.2, 0.02, 10000, direction=-1)
    assert len(laps.crossing_times(laps.lap_progress(X, TRACK, 1), 0.02)) == 0


def test_backtracking_does_not_recount():
    # forward past one lap, back below it, forward again: the lap is counted once
    dt = 0.02
    phi = np.concatenate([np.linspace(0, 2 * np.pi * 1.05, 500), np.linspace(2 * np.pi * 1.05, 2 * np.pi * 0.9, 100),
                          np.linspace(2 * np.pi * 0.9, 2 * np.pi * 1.5, 300)])
    (cx, cy), (a, b) = TRACK.center, TRACK.semi_axes
    X = np.zeros((len(phi), 7))
    X[:, 0], X[:, 1] = cx + a * np.cos(phi), cy + b * np.sin(phi)
    assert len(laps.crossing_times(laps.lap_progress(X, TRACK, 1), dt)) == 1


def test_classification_and_statistics():
    dt, omega = 0.02, 2 * math.pi / 10.0          # 10 s laps, 500 steps each
    X = _ellipse_traj(0.0, omega, dt, 5 * 500 + 10)
    h = np.zeros(len(X))
    h[2 * 500 + 123] = 1.0                          # off the track during the third lap
    m = laps.lap_metrics(X, h, dt, TRACK, 1, crash_threshold=0.99)
    # five complete laps, the first discarded: four counted, one of them failed
    assert m["laps"] == 4 and m["success_pct"] == 75.0
    assert [l["success"] for l in m["per_lap"]] == [True, True, False, True, True]
    np.testing.assert_allclose(m["lap_time_mean"], 10.0, rtol=1e-6)
    assert m["lap_time_std"] < 1e-6
    assert 4.89 < m["speed_min"] < 4.91 and 5.09 < m["speed_max"] < 5.11
    # non-finite states fail their lap too
    X2 = X.copy()
    X2[4 * 500 + 7, 5] = np.nan
    m2 = laps.lap_metrics(X2, h, dt, TRACK, 1, crash_threshold=0.99)
    assert [l["success"] for l in m2["per_lap"]] == [True, True, False, True, False]
