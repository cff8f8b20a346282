"""Seeded synthetic inputs shared by the GPU library's tests/bench and the CPU oracle.

This module holds no arithmetic of the MPPI method itself: it only draws the
inputs the method consumes (costmaps, dynamics-network parameters, initial
states, problem parameters).  The paper's own inputs (a GPS-surveyed dirt
track turned into a spline cost map, Section VI-C; a network trained on a
30-minute driving dataset, Section VI-B) are not available, so every input
here is a synthetic stand-in with the shapes the paper describes:

* cost maps with values in [0, 1] that are 0 on the track and rise to 1 past
  its boundary (the paper's map is |spline| with +-1 on the boundaries,
  capped at 2.5; Section VI-C "Track Cost");
* a 6 -> h -> h -> 4 tanh network (h = 32 gives the paper's 1412 parameters,
  Section VI-B-2) with Xavier-uniform weights and zero biases;
* vehicle states (p_x, p_y, theta, roll, v_x, v_y, theta_dot) (Section VI-B).

All floating-point inputs are generated in float64 and rounded once to float32;
both sides receive the identical float32 arrays.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

N_STATE = 7
N_CTRL = 2
MLP_IN = 6
MLP_OUT = 4


# ----------------------------------------------------------------------------
# Dynamics network parameters
# ----------------------------------------------------------------------------

def mlp_param_count(hidden: int) -> int:
    """Packed parameter count of the 6 -> h -> h -> 4 network (W1,b1,W2,b2,W3,b3)."""
    return MLP_IN * hidden + hidden + hidden * hidden + hidden + MLP_OUT * hidden + MLP_OUT


def mlp_params(hidden: int = 32, seed: int = 0, bias_scale: float = 0.0) -> np.ndarray:
    """Xavier-uniform weights (+-sqrt(6/(fan_in+fan_out))), zero biases by default.

    Packing (float32, row-major [out][in]): W1[h][6], b1[h], W2[h][h], b2[h],
    W3[4][h], b3[4].
    """
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((MLP_IN, hidden), (hidden, hidden), (hidden, MLP_OUT)):
        bound = math.sqrt(6.0 / (fan_in + fan_out))
        w = rng.uniform(-bound, bound, size=(fan_out, fan_in))
        b = rng.uniform(-bias_scale, bias_scale, size=(fan_out,)) if bias_scale > 0 else np.zeros(fan_out)
        parts += [w.ravel(), b]
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == mlp_param_count(hidden)
    return out


# Basis-function model (appendix): Theta is [25][4], row i for basis function i + 1,
# column o for d/dt of (roll, v_x, v_y, heading rate).  No system-identification data is
# available, so Theta is synthetic: a damped, steerable base written in the appendix's
# own terms (throttle drives v_x against linear and quadratic drag, the front and rear
# tyre terms tan(alpha) drive v_y and the heading rate, rates are damped, roll relaxes)
# plus seeded N(0, noise^2) entries scaled by each basis function's normaliser, so that
# every basis function contributes.  The drag polynomial of v_x (basis functions 2, 22,
# 23 in the v_x column) carries no noise, so that the top speed stays set by throttle
# and drag (about 11 m/s at full throttle).
N_BASIS = 25
_BASIS_NORM = [1.0, 10.0, 1200.0, 1200.0 ** 2, 1200.0 ** 3, 25.0, 10.0, 10.0, 1.0, 40.0, 1400.0,
               1400.0 ** 2, 1400.0 ** 3, 40.0, 40.0 ** 2, 40.0 ** 3, 50.0, 1.0, 1.0, 3.0, 5.0, 100.0,
               1000.0, 1.0, 1.0]
# (basis function number, output, coefficient of the basis function times its normaliser,
# e.g. -0.3 on v_x for basis 2 = v_x / 10)
_BASIS_BASE = [(18, 0, -4.0), (17, 0, 0.04),
               (1, 1, 6.0), (2, 1, -0.3), (22, 1, -0.02), (6, 1, 1.0),
               (17, 2, -1.0), (8, 2, -2.0), (11, 2, -4.0), (14, 2, -3.0),
               (11, 3, -5.0), (14, 3, 3.0), (7, 3, -1.0)]
_BASIS_QUIET = [(2, 1), (22, 1), (23, 1)]


def basis_theta(seed: int = 0, noise: float = 0.05) -> np.ndarray:
    """A synthetic Theta [25][4] (float32, row-major) for the basis-function model."""
    rng = np.random.default_rng(20_000 + seed)
    norm = np.array(_BASIS_NORM)[:, None]
    theta = noise * rng.standard_normal((N_BASIS, 4)) * norm
    for i, o in _BASIS_QUIET:
        theta[i - 1, o] = 0.0
    for i, o, c in _BASIS_BASE:
        theta[i - 1, o] += c * _BASIS_NORM[i - 1]
    return theta.astype(np.float32)


def mlp_unpack(params: np.ndarray, hidden: int):
    """Split a packed parameter vector into (W1, b1, W2, b2, W3, b3) views."""
    h = hidden
    sizes = [(h, MLP_IN), (h,), (h, h), (h,), (MLP_OUT, h), (MLP_OUT,)]
    out, off = [], 0
    for s in sizes:
        n = int(np.prod(s))
        out.append(params[off:off + n].reshape(s))
        off += n
    assert off == params.size
    return out


# ----------------------------------------------------------------------------
# Cost maps
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class CostMap:
    data: np.ndarray          # [H][W] float32, row i = y, column j = x
    origin_x: float           # world x of cell (i, j=0)
    origin_y: float           # world y of cell (i=0, j)
    resolution: float         # metres per cell

    @property
    def H(self) -> int:
        return int(self.data.shape[0])

    @property
    def W(self) -> int:
        return int(self.data.shape[1])


def _blur_clamp(mask: np.ndarray, sigma_cells: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    out = gaussian_filter(mask.astype(np.float64), sigma=sigma_cells, mode="reflect")
    return np.clip(out, 0.0, 1.0).astype(np.float32)


@functools.lru_cache(maxsize=4)
def ring_map(H: int = 256, W: int = 256, resolution: float = 0.1,
             center=(12.8, 12.8), radius: float = 8.0, half_width: float = 2.0,
             blur_sigma_cells: float = 2.0) -> CostMap:
    """Circular ring track: 0 within half_width of the centre-line circle, 1 outside,
    then Gaussian-blurred (reflect padding) and clamped to [0, 1]."""
    res = np.float32(resolution)
    ys = (np.arange(H) * float(res))[:, None]
    xs = (np.arange(W) * float(res))[None, :]
    d = np.hypot(xs - center[0], ys - center[1]) - radius
    mask = (np.abs(d) > half_width).astype(np.float64)
    data = _blur_clamp(mask, blur_sigma_cells)
    data.setflags(write=False)
    return CostMap(data, 0.0, 0.0, float(res))


def _ellipse_distance(px: np.ndarray, py: np.ndarray, cx: float, cy: float, a: float, b: float,
                      iters: int = 12) -> np.ndarray:
    """Unsigned distance from points to the ellipse (cx + a cos phi, cy + b sin phi): Newton
    on the stationarity condition of |curve(phi) - p|^2 from three starting angles, keeping
    the nearest stationary point found."""
    x = (px - cx).astype(np.float64)
    y = (py - cy).astype(np.float64)
    base = np.arctan2(a * y, b * x)
    best = np.full(x.shape, np.inf)
    for off in (0.0, 0.35, -0.35):
        phi = base + off
        for _ in range(iters):
            c, s = np.cos(phi), np.sin(phi)
            f = (a * a - b * b) * s * c - x * a * s + y * b * c
            df = (a * a - b * b) * (c * c - s * s) - x * a * c - y * b * s
            step = np.where(np.abs(df) > 1e-12, f / np.where(df == 0, 1.0, df), 0.0)
            phi = phi - np.clip(step, -0.5, 0.5)
        d = np.hypot(a * np.cos(phi) - x, b * np.sin(phi) - y)
        best = np.minimum(best, d)
    return best


@functools.lru_cache(maxsize=2)
def ellipse_map(H: int = 2048, W: int = 2048, resolution: float = 0.05,
                center=(51.2, 51.2), semi_axes=(40.0, 25.0), half_width: float = 5.0,
                blur_sigma_cells: float = 5.0) -> CostMap:
    """Closed elliptical track 2*half_width wide around an elliptical centre line;
    walls blurred with a Gaussian (reflect) and clamped to [0, 1]."""
    res = np.float32(resolution)
    ys, xs = np.meshgrid(np.arange(H) * float(res), np.arange(W) * float(res), indexing="ij")
    a, b = semi_axes
    # A point at scaled-ellipse coordinate r lies at least |r - 1| * min(a, b) from the curve,
    # so only the band |r - 1| <= (half_width + 1) / min(a, b) needs the distance solve.
    r = np.hypot((xs - center[0]) / a, (ys - center[1]) / b)
    band = np.abs(r - 1.0) <= (half_width + 1.0) / min(a, b)
    d = np.full(xs.shape, np.inf)
    d[band] = _ellipse_distance(xs[band], ys[band], center[0], center[1], a, b)
    mask = (d > half_width).astype(np.float64)
    data = _blur_clamp(mask, blur_sigma_cells)
    data.setflags(write=False)
    return CostMap(data, 0.0, 0.0, float(res))


def constant_map(value: float, H: int = 64, W: int = 64, resolution: float = 0.5,
                 origin=(0.0, 0.0)) -> CostMap:
    data = np.full((H, W), value, dtype=np.float32)
    return CostMap(data, float(np.float32(origin[0])), float(np.float32(origin[1])),
                   float(np.float32(resolution)))


def affine_map(a: float, b: float, c: float, H: int = 64, W: int = 64, resolution: float = 0.5,
               origin=(0.0, 0.0)) -> CostMap:
    """m[i][j] = a + b*i + c*j (rounded to float32)."""
    i = np.arange(H, dtype=np.float64)[:, None]
    j = np.arange(W, dtype=np.float64)[None, :]
    data = (a + b * i + c * j).astype(np.float32)
    return CostMap(data, float(np.float32(origin[0])), float(np.float32(origin[1])),
                   float(np.float32(resolution)))


def split_nan_map(x_max: np.ndarray, y_center: float, value: float = 0.25, resolution: float = 0.002,
                  size: int = 2048):
    """A constant map whose columns beyond a boundary are NaN, placed so that about half of
    the samples, given the largest x each reaches (x_max, from a rollout), read a NaN cell
    and the others do not.  The boundary grid line sits in the middle of the widest gap
    between consecutive sorted x_max values in their middle third, and 1000 cells from
    the map's left edge; lookups at x >= boundary touch the NaN column.  Returns the map
    and the width of that gap."""
    xs = np.sort(np.asarray(x_max, np.float64))
    lo, hi = len(xs) // 3, max(len(xs) * 2 // 3, len(xs) // 3 + 1)
    gaps = xs[lo + 1:hi + 1] - xs[lo:hi]
    i = lo + int(np.argmax(gaps))
    boundary = 0.5 * (xs[i] + xs[i + 1])
    res = float(np.float32(resolution))
    ox = float(np.float32(boundary - 1000 * res))
    oy = float(np.float32(y_center - 0.5 * size * res))
    data = np.full((size, size), value, dtype=np.float32)
    data[:, 1001:] = np.nan
    return CostMap(data, ox, oy, res), float(xs[i + 1] - xs[i])


# ----------------------------------------------------------------------------
# Problem parameters
# ----------------------------------------------------------------------------

@dataclass
class CostParams:
    """State cost c(x, t):  w_map*h + crash_cost*crash_decay^t*[h > map_thresh]
    + w_speed*(v_x - v_des)^2 + w_slip*zeta^2 + slip_cost*[|zeta| > slip_thresh],
    zeta = -atan2(v_y, |v_x|)."""
    w_map: float = 100.0
    w_speed: float = 1.0
    w_slip: float = 0.0
    v_des: float = 6.0
    crash_cost: float = 0.0
    crash_decay: float = 1.0
    map_thresh: float = float("inf")
    slip_cost: float = 0.0
    slip_thresh: float = float("inf")


@dataclass
class Problem:
    K: int
    T: int
    hidden: int = 32
    dt: float = 0.02
    lam: float = 1.0
    gamma: Optional[float] = None        # None -> gamma = lambda
    sigma2: tuple = (0.3, 0.35)          # covariance diagonal (variances)
    u_lo: tuple = (-1.0, -1.0)
    u_hi: tuple = (1.0, 1.0)
    sg_window: int = 1
    sg_order: int = 0
    seed: int = 0
    instance: int = 0
    explore: float = 0.0                 # fraction of zero-mean (exploration) samples
    model: int = 0                       # 0: network (params = packed MLP), 1: basis functions (Theta)
    weighting: int = 0                   # 0: Algorithm 2 (information theoretic), 1: Algorithm 3 (CEM)
    elite: float = 0.8                   # Algorithm 3's eliteness threshold (percentile)
    cost: CostParams = field(default_factory=CostParams)
    k_base: int = 0                      # K-shard form: global index of this shard's sample 0
    k_total: int = 0                     # K-shard form: samples of the whole iteration (0: unsharded)

    @property
    def gamma_value(self) -> float:
        return self.lam if self.gamma is None else self.gamma


# ----------------------------------------------------------------------------
# The five workload shapes
# ----------------------------------------------------------------------------

C1_X0 = np.array([20.8, 12.8, math.pi / 2, 0.0, 4.0, 0.0, 0.0], dtype=np.float32)
C2_X0 = np.array([91.2, 51.2, math.pi / 2, 0.0, 4.0, 0.0, 0.0], dtype=np.float32)


def c1_problem(seed: int = 0) -> Problem:
    """Plain MPPI: K=256, T=30, ring map, cost 100*h + (v_x-6)^2, lambda=1, SGF off."""
    return Problem(K=256, T=30, hidden=32, dt=0.02, lam=1.0, sigma2=(0.3, 0.35),
                   sg_window=1, sg_order=0, seed=seed,
                   cost=CostParams(w_map=100.0, w_speed=1.0, v_des=6.0))


def c2_cost() -> CostParams:
    return CostParams(w_map=100.0, w_speed=1.0, w_slip=1.0, v_des=8.0,
                      crash_cost=1.0e4, crash_decay=0.9, map_thresh=0.99,
                      slip_cost=1.0e4, slip_thresh=0.75)


def c2_problem(seed: int = 0) -> Problem:
    """Paper-shaped: K=1920, T=100, elliptical 2048^2 map, speed 8 m/s, slip and crash
    impulses, lambda=6.7, Savitzky-Golay window 9 / order 2."""
    return Problem(K=1920, T=100, hidden=32, dt=0.02, lam=6.7, sigma2=(0.3, 0.35),
                   sg_window=9, sg_order=2, seed=seed, cost=c2_cost())


def c3_problem(K: int = 16384, seed: int = 0) -> Problem:
    """Precision form: hidden 64, T=100, C1's map and cost."""
    return Problem(K=K, T=100, hidden=64, dt=0.02, lam=1.0, sigma2=(0.3, 0.35),
                   sg_window=1, sg_order=0, seed=seed,
                   cost=CostParams(w_map=100.0, w_speed=1.0, v_des=6.0))


def c5_problem(seed: int = 0) -> Problem:
    """Differentiation form: K=4096, T=100, hidden 32, C1's smooth cost."""
    return Problem(K=4096, T=100, hidden=32, dt=0.02, lam=1.0, sigma2=(0.3, 0.35),
                   sg_window=1, sg_order=0, seed=seed,
                   cost=CostParams(w_map=100.0, w_speed=1.0, v_des=6.0))


def basis_problem(seed: int = 0, K: int = 1920) -> Problem:
    """The paper-shaped problem (K=1920, T=100, elliptical map, impulses, SGF 9/2) with the
    basis-function model in place of the network (params = basis_theta())."""
    return replace(c2_problem(seed), K=K, model=1)


def explore_problem(seed: int = 0, K: int = 1920, explore: float = 0.01) -> Problem:
    """Exploration samples with the paper's parameter table: the paper-shaped C2 problem
    with lambda=12.5, gamma=0.1, Sigma=Diag(0.0306, 0.0506) (variances) and a fraction
    alpha=0.01 of zero-mean samples."""
    return Problem(K=K, T=100, hidden=32, dt=0.02, lam=12.5, gamma=0.1, sigma2=(0.0306, 0.0506),
                   sg_window=9, sg_order=2, seed=seed, explore=explore, cost=c2_cost())


def cem_problem(seed: int = 0, K: int = 1920, elite: float = 0.8) -> Problem:
    """Cross-entropy weights (Algorithm 3) on the parameter-table problem: the top
    20 % of the samples (eliteness threshold 0.8), no exploration samples."""
    return replace(explore_problem(seed, K=K, explore=0.0), weighting=1, elite=elite)


def ellipse_pose(phi: float, v_x: float, center=(51.2, 51.2), semi_axes=(40.0, 25.0)) -> np.ndarray:
    """A pose on the elliptical centre line at parameter phi, heading along the
    counter-clockwise tangent, with forward speed v_x and other states 0."""
    a, b = semi_axes
    x = center[0] + a * math.cos(phi)
    y = center[1] + b * math.sin(phi)
    heading = math.atan2(b * math.cos(phi), -a * math.sin(phi))
    return np.array([x, y, heading, 0.0, v_x, 0.0, 0.0], dtype=np.float32)


@dataclass
class BatchInstance:
    K: int
    T: int
    x0: np.ndarray


def c4_instances(n: int = 512, seed: int = 0) -> list:
    """Batched form: K_i ~ U{512,1024,2048,4096}, T_i ~ U{50,75,100,150}, start poses on
    the elliptical centre line with v_x ~ U[2,10]."""
    rng = np.random.default_rng(seed)
    Ks = rng.choice([512, 1024, 2048, 4096], size=n)
    Ts = rng.choice([50, 75, 100, 150], size=n)
    phis = rng.uniform(0.0, 2.0 * math.pi, size=n)
    vxs = rng.uniform(2.0, 10.0, size=n)
    return [BatchInstance(int(Ks[i]), int(Ts[i]), ellipse_pose(float(phis[i]), float(vxs[i])))
            for i in range(n)]


def random_controls(T: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """A nominal control sequence [T][2] for tests that start away from zero."""
    rng = np.random.default_rng(10_000 + seed)
    return (scale * rng.standard_normal((T, N_CTRL))).astype(np.float32)


def with_(p: Problem, **kw) -> Problem:
    return replace(p, **kw)
