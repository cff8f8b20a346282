"""Thin ctypes binding of libmppi.so (include/mppi.h): argument marshalling only.

Every computation of the MPPI iteration runs in the library's HIP kernels.
There is no CPU fallback: if the library is not built, loading fails loudly.
PyTorch is used, when present, only to hand the library a HIP stream.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path
from typing import Optional

import numpy as np

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "libmppi.so"

MPPI_OK, MPPI_E_INVAL, MPPI_E_STATE, MPPI_E_NOMEM, MPPI_E_DEVICE, MPPI_E_NONFINITE = range(6)
MPPI_PREC_FP32, MPPI_PREC_BF16, MPPI_PREC_FP16 = 0, 1, 2
MPPI_SCHED_AUTO, MPPI_SCHED_LANE, MPPI_SCHED_WAVE, MPPI_SCHED_WIDE, MPPI_SCHED_QUAD = 0, 1, 2, 3, 4
MPPI_WEIGHTS_IT, MPPI_WEIGHTS_CEM = 0, 1
MPPI_T_MAX = 256

STATUS_NAMES = {0: "MPPI_OK", 1: "MPPI_E_INVAL", 2: "MPPI_E_STATE", 3: "MPPI_E_NOMEM",
                4: "MPPI_E_DEVICE", 5: "MPPI_E_NONFINITE"}

# Every function the header declares; tests check that the library exports each.
EXPORTED = [
    "mppi_create", "mppi_destroy", "mppi_last_error", "mppi_set_costmap", "mppi_set_dynamics",
    "mppi_set_basis_dynamics", "mppi_costmap_values",
    "mppi_set_controls", "mppi_iterate", "mppi_iterate_device", "mppi_get_controls", "mppi_shift",
    "mppi_plant_step", "mppi_run_receding", "mppi_step_device", "mppi_get_stats", "mppi_get_noise",
    "mppi_get_iteration", "mppi_set_iteration", "mppi_get_schedule", "mppi_set_timing",
    "mppi_get_timing", "mppi_get_timing_samples", "mppi_objective", "mppi_objective_backward",
    "mppi_batch_create", "mppi_batch_destroy", "mppi_batch_last_error", "mppi_batch_set_costmap",
    "mppi_batch_set_dynamics", "mppi_batch_set_controls", "mppi_batch_iterate",
    "mppi_batch_get_controls", "mppi_batch_get_costs", "mppi_batch_get_schedule",
    "mppi_batch_synchronize", "mppi_iterate_noalloc", "mppi_iterate_partial", "mppi_merge_update",
    "mppi_run_receding_device",
]


class mppi_config(C.Structure):
    _fields_ = [("K", C.c_int32), ("T", C.c_int32), ("dt", C.c_float), ("lam", C.c_float),
                ("gamma", C.c_float), ("sigma2", C.c_float * 2), ("u_lo", C.c_float * 2),
                ("u_hi", C.c_float * 2), ("sg_window", C.c_int32), ("sg_order", C.c_int32),
                ("precision", C.c_int32), ("schedule", C.c_int32), ("seed", C.c_uint64),
                ("instance", C.c_uint32), ("explore", C.c_float), ("weighting", C.c_int32),
                ("elite", C.c_float), ("k_base", C.c_uint32), ("k_total", C.c_int32)]


class mppi_cost(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("w_map", "w_speed", "w_slip", "v_des", "crash_cost",
                                         "crash_decay", "map_thresh", "slip_cost", "slip_thresh")]


class MppiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """Load libmppi.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is not built; run paper_1707_02342_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(str(LIB_PATH))
        vp = C.c_void_p
        fp = C.POINTER(C.c_float)
        L.mppi_create.argtypes = [C.POINTER(mppi_config), C.POINTER(mppi_cost), C.c_int, vp, C.POINTER(vp)]
        L.mppi_destroy.argtypes = [vp]
        L.mppi_destroy.restype = None
        L.mppi_last_error.argtypes = [vp]
        L.mppi_last_error.restype = C.c_char_p
        L.mppi_set_costmap.argtypes = [vp, fp, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float]
        L.mppi_set_dynamics.argtypes = [vp, C.POINTER(C.c_int32), fp]
        L.mppi_set_basis_dynamics.argtypes = [vp, fp]
        L.mppi_costmap_values.argtypes = [vp, fp, C.c_int32, fp]
        L.mppi_set_controls.argtypes = [vp, fp]
        L.mppi_iterate.argtypes = [vp, fp, fp]
        L.mppi_iterate_device.argtypes = [vp, vp]
        L.mppi_get_controls.argtypes = [vp, fp]
        L.mppi_shift.argtypes = [vp, fp]
        L.mppi_plant_step.argtypes = [vp, fp, fp, fp]
        L.mppi_run_receding.argtypes = [vp, fp, C.c_int32, fp, fp]
        L.mppi_step_device.argtypes = [vp, vp, vp]
        L.mppi_get_stats.argtypes = [vp, fp, fp, fp]
        L.mppi_get_noise.argtypes = [vp, C.c_uint32, fp]
        L.mppi_get_iteration.argtypes = [vp, C.POINTER(C.c_uint32)]
        L.mppi_set_iteration.argtypes = [vp, C.c_uint32]
        L.mppi_get_schedule.argtypes = [vp, C.POINTER(C.c_int32)]
        L.mppi_set_timing.argtypes = [vp, C.c_int32]
        L.mppi_get_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.mppi_get_timing_samples.argtypes = [vp, fp, C.c_int32, C.POINTER(C.c_int32)]
        L.mppi_objective.argtypes = [vp, fp, C.c_uint32, C.c_int32, C.POINTER(C.c_double), fp]
        L.mppi_objective_backward.argtypes = [vp, fp, fp]
        i32p = C.POINTER(C.c_int32)
        L.mppi_batch_create.argtypes = [C.POINTER(mppi_config), C.POINTER(mppi_cost), C.c_int32, i32p, i32p,
                                        C.c_int, vp, C.POINTER(vp)]
        L.mppi_batch_destroy.argtypes = [vp]
        L.mppi_batch_destroy.restype = None
        L.mppi_batch_last_error.argtypes = [vp]
        L.mppi_batch_last_error.restype = C.c_char_p
        L.mppi_batch_set_costmap.argtypes = [vp, fp, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float]
        L.mppi_batch_set_dynamics.argtypes = [vp, i32p, fp]
        L.mppi_batch_set_controls.argtypes = [vp, C.c_int32, fp]
        L.mppi_batch_iterate.argtypes = [vp, fp]
        L.mppi_batch_get_controls.argtypes = [vp, C.c_int32, fp]
        L.mppi_batch_get_costs.argtypes = [vp, C.c_int32, fp]
        L.mppi_batch_get_schedule.argtypes = [vp, i32p, i32p, C.POINTER(C.c_double), i32p]
        L.mppi_batch_synchronize.argtypes = [vp]
        L.mppi_iterate_partial.argtypes = [vp, fp, vp, fp]
        L.mppi_run_receding_device.argtypes = [vp, vp, C.c_int32, vp, vp]
        L.mppi_merge_update.argtypes = [vp, vp, C.c_int32]
        L.mppi_iterate_noalloc.argtypes = [C.POINTER(mppi_config), C.POINTER(mppi_cost), C.c_int, vp, vp,
                                           C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float, i32p, vp, vp,
                                           C.c_uint32, vp, vp, vp]
        for name in EXPORTED:
            if name not in ("mppi_destroy", "mppi_last_error", "mppi_batch_destroy", "mppi_batch_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _f32(a, shape=None) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None and out.shape != tuple(shape):
        out = out.reshape(shape)
    return out


def _fp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_float))


# ---------------------------------------------------------------------------
# Same-named wrappers of the C entry points
# ---------------------------------------------------------------------------

def _check(ctx, st: int, allow=(MPPI_OK,)) -> int:
    if st not in allow:
        raise MppiError(st, mppi_last_error(ctx))
    return st


def mppi_last_error(ctx) -> str:
    r = lib().mppi_last_error(ctx)
    return r.decode() if r else ""


def mppi_create(cfg: mppi_config, cost: mppi_cost, device: int = 0, stream: int = 0):
    out = C.c_void_p()
    st = lib().mppi_create(C.byref(cfg), C.byref(cost), device, C.c_void_p(stream or None), C.byref(out))
    if st != MPPI_OK:
        raise MppiError(st, mppi_last_error(None))
    return out


def mppi_destroy(ctx) -> None:
    lib().mppi_destroy(ctx)


def mppi_set_costmap(ctx, data, origin_x: float, origin_y: float, resolution: float) -> None:
    m = _f32(data)
    _check(ctx, lib().mppi_set_costmap(ctx, _fp(m), m.shape[0], m.shape[1], origin_x, origin_y, resolution))


def mppi_set_dynamics(ctx, hidden: int, params) -> None:
    dims = (C.c_int32 * 4)(6, hidden, hidden, 4)
    p = _f32(params)
    _check(ctx, lib().mppi_set_dynamics(ctx, dims, _fp(p)))


def mppi_set_basis_dynamics(ctx, theta) -> None:
    t = _f32(theta).reshape(-1)
    if t.size != 100:
        raise ValueError("Theta must hold 25 x 4 entries")
    _check(ctx, lib().mppi_set_basis_dynamics(ctx, _fp(t)))


def mppi_costmap_values(ctx, xy) -> np.ndarray:
    p = _f32(xy).reshape(-1, 2)
    h = np.zeros(p.shape[0], dtype=np.float32)
    _check(ctx, lib().mppi_costmap_values(ctx, _fp(p), p.shape[0], _fp(h)))
    return h


def mppi_set_controls(ctx, U) -> None:
    u = _f32(U)
    _check(ctx, lib().mppi_set_controls(ctx, _fp(u)))


def mppi_iterate(ctx, x0, costs_out: Optional[np.ndarray] = None) -> int:
    x = _f32(x0)
    return _check(ctx, lib().mppi_iterate(ctx, _fp(x), _fp(costs_out)), allow=(MPPI_OK, MPPI_E_NONFINITE))


def mppi_iterate_device(ctx, x0_dev_ptr: int) -> None:
    _check(ctx, lib().mppi_iterate_device(ctx, C.c_void_p(x0_dev_ptr)))


def mppi_get_controls(ctx, T: int):
    U = np.zeros((T, 2), dtype=np.float32)
    st = _check(ctx, lib().mppi_get_controls(ctx, _fp(U)), allow=(MPPI_OK, MPPI_E_NONFINITE))
    return U, st


def mppi_shift(ctx):
    u0 = np.zeros(2, dtype=np.float32)
    st = _check(ctx, lib().mppi_shift(ctx, _fp(u0)), allow=(MPPI_OK, MPPI_E_NONFINITE))
    return u0, st


def mppi_plant_step(ctx, x, u):
    xi = _f32(x)
    ui = _f32(u)
    xo = np.zeros(7, dtype=np.float32)
    _check(ctx, lib().mppi_plant_step(ctx, _fp(xi), _fp(ui), _fp(xo)))
    return xo


def mppi_run_receding(ctx, x0, n_iter: int):
    x = _f32(x0)
    uh = np.zeros((n_iter, 2), dtype=np.float32)
    xh = np.zeros((n_iter + 1, 7), dtype=np.float32)
    st = _check(ctx, lib().mppi_run_receding(ctx, _fp(x), n_iter, _fp(uh), _fp(xh)),
                allow=(MPPI_OK, MPPI_E_NONFINITE))
    return uh, xh, st


def mppi_step_device(ctx, x_dev_ptr: int, u0_dev_ptr: int = 0) -> None:
    """One receding-horizon step on device data (pointers as integers, e.g. data_ptr())."""
    _check(ctx, lib().mppi_step_device(ctx, C.c_void_p(x_dev_ptr), C.c_void_p(u0_dev_ptr or None)))


def mppi_iterate_partial(ctx, x0, row_dev_ptr: int, costs_out: Optional[np.ndarray] = None) -> None:
    """K-shard form: one iteration of this context's samples whose merged row
    (rho_g, eta_g, N_g[T][2]) goes to the device buffer at row_dev_ptr ([2 + 2T] floats);
    the shard's costs into costs_out when given."""
    x = _f32(x0)
    _check(ctx, lib().mppi_iterate_partial(ctx, _fp(x), C.c_void_p(row_dev_ptr), _fp(costs_out)))


def mppi_merge_update(ctx, rows_dev_ptr: int, n_rows: int) -> None:
    """K-shard form: merge n_rows shard rows ([n_rows][2 + 2T] on the device) and update U."""
    _check(ctx, lib().mppi_merge_update(ctx, C.c_void_p(rows_dev_ptr), n_rows))


def mppi_run_receding_device(ctx, x_dev_ptr: int, n_iter: int, u_hist_dev_ptr: int = 0,
                             x_hist_dev_ptr: int = 0) -> None:
    """n_iter receding steps on device data (pointers as integers); enqueued."""
    _check(ctx, lib().mppi_run_receding_device(ctx, C.c_void_p(x_dev_ptr), n_iter, C.c_void_p(u_hist_dev_ptr or None),
                                               C.c_void_p(x_hist_dev_ptr or None)))


def mppi_get_stats(ctx, T: int):
    rho, eta = C.c_float(), C.c_float()
    d = np.zeros((T, 2), dtype=np.float32)
    _check(ctx, lib().mppi_get_stats(ctx, C.byref(rho), C.byref(eta), _fp(d)))
    return rho.value, eta.value, d


def mppi_get_noise(ctx, it: int, K: int, T: int):
    e = np.zeros((K, T, 2), dtype=np.float32)
    _check(ctx, lib().mppi_get_noise(ctx, it, _fp(e)))
    return e


def mppi_get_iteration(ctx) -> int:
    v = C.c_uint32()
    _check(ctx, lib().mppi_get_iteration(ctx, C.byref(v)))
    return v.value


def mppi_set_iteration(ctx, it: int) -> None:
    _check(ctx, lib().mppi_set_iteration(ctx, it))


def mppi_get_schedule(ctx) -> int:
    v = C.c_int32()
    _check(ctx, lib().mppi_get_schedule(ctx, C.byref(v)))
    return v.value


def mppi_set_timing(ctx, enable: bool) -> None:
    _check(ctx, lib().mppi_set_timing(ctx, 1 if enable else 0))


def mppi_get_timing(ctx):
    t = (C.c_double * 2)()
    n = (C.c_int64 * 2)()
    _check(ctx, lib().mppi_get_timing(ctx, t, n))
    return (t[0], t[1]), (n[0], n[1])


def mppi_get_timing_samples(ctx, cap: int = 1 << 16) -> np.ndarray:
    """Per-launch kernel durations (ms) recorded since timing was enabled."""
    buf = np.zeros(cap, dtype=np.float32)
    n = C.c_int32()
    _check(ctx, lib().mppi_get_timing_samples(ctx, _fp(buf), cap, C.byref(n)))
    return buf[:min(n.value, cap)].copy()


def mppi_objective(ctx, x0, it: int, ckpt_every: int = 10, K: Optional[int] = None):
    x = _f32(x0)
    J = C.c_double()
    S = np.zeros(K, dtype=np.float32) if K else None
    _check(ctx, lib().mppi_objective(ctx, _fp(x), it, ckpt_every, C.byref(J), _fp(S)))
    return J.value, S


def mppi_objective_backward(ctx, T: int, n_params: int = 1412):
    gU = np.zeros((T, 2), dtype=np.float32)
    gth = np.zeros(n_params, dtype=np.float32)
    _check(ctx, lib().mppi_objective_backward(ctx, _fp(gU), _fp(gth)))
    return gU, gth


def mppi_batch_last_error(b) -> str:
    r = lib().mppi_batch_last_error(b)
    return r.decode() if r else ""


def _bcheck(b, st: int, allow=(MPPI_OK,)) -> int:
    if st not in allow:
        raise MppiError(st, mppi_batch_last_error(b))
    return st


def mppi_batch_create(cfg: mppi_config, cost: mppi_cost, Ks, Ts, device: int = 0, stream: int = 0):
    K = np.ascontiguousarray(Ks, dtype=np.int32)
    T = np.ascontiguousarray(Ts, dtype=np.int32)
    out = C.c_void_p()
    st = lib().mppi_batch_create(C.byref(cfg), C.byref(cost), K.size, K.ctypes.data_as(C.POINTER(C.c_int32)),
                                 T.ctypes.data_as(C.POINTER(C.c_int32)), device, C.c_void_p(stream or None),
                                 C.byref(out))
    if st != MPPI_OK:
        raise MppiError(st, mppi_batch_last_error(None))
    return out


def mppi_batch_destroy(b) -> None:
    lib().mppi_batch_destroy(b)


def mppi_batch_set_costmap(b, data, origin_x, origin_y, resolution) -> None:
    m = _f32(data)
    _bcheck(b, lib().mppi_batch_set_costmap(b, _fp(m), m.shape[0], m.shape[1], origin_x, origin_y, resolution))


def mppi_batch_set_dynamics(b, params) -> None:
    dims = (C.c_int32 * 4)(6, 32, 32, 4)
    p = _f32(params)
    _bcheck(b, lib().mppi_batch_set_dynamics(b, dims, _fp(p)))


def mppi_batch_set_controls(b, i: int, U) -> None:
    u = _f32(U)
    _bcheck(b, lib().mppi_batch_set_controls(b, i, _fp(u)))


def mppi_batch_iterate(b, x0) -> None:
    x = _f32(x0)
    _bcheck(b, lib().mppi_batch_iterate(b, _fp(x)))


def mppi_batch_get_controls(b, i: int, T: int):
    U = np.zeros((T, 2), dtype=np.float32)
    st = _bcheck(b, lib().mppi_batch_get_controls(b, i, _fp(U)), allow=(MPPI_OK, MPPI_E_NONFINITE))
    return U, st


def mppi_batch_get_costs(b, i: int, K: int):
    S = np.zeros(K, dtype=np.float32)
    _bcheck(b, lib().mppi_batch_get_costs(b, i, _fp(S)))
    return S


def mppi_batch_get_schedule(b):
    """(grid, order, tuned_us, schedule) the autotuner chose."""
    g, o, t, s = C.c_int32(), C.c_int32(), C.c_double(), C.c_int32()
    _bcheck(b, lib().mppi_batch_get_schedule(b, C.byref(g), C.byref(o), C.byref(t), C.byref(s)))
    return g.value, o.value, t.value, s.value


def mppi_batch_synchronize(b) -> None:
    _bcheck(b, lib().mppi_batch_synchronize(b))


def mppi_iterate_noalloc(cfg: mppi_config, cost: mppi_cost, device: int, stream: int, map_dev: int, H: int,
                         W: int, origin_x: float, origin_y: float, resolution: float, hidden: int,
                         params_dev: int, x0_dev: int, it: int, U_dev: int, S_dev: int = 0,
                         status_dev: int = 0) -> None:
    """One context-free iteration on device buffers (pointers as integers, e.g.
    data_ptr()); nothing is allocated.  Errors raise with mppi_last_error(NULL)."""
    dims = (C.c_int32 * 4)(6, hidden, hidden, 4)
    vp = C.c_void_p
    st = lib().mppi_iterate_noalloc(C.byref(cfg), C.byref(cost), device, vp(stream or None), vp(map_dev), H, W,
                                    origin_x, origin_y, resolution, dims, vp(params_dev), vp(x0_dev), it,
                                    vp(U_dev), vp(S_dev or None), vp(status_dev or None))
    if st != MPPI_OK:
        raise MppiError(st, mppi_last_error(None))


class Batch:
    """Many MPPI problems advanced by one persistent launch (see mppi_batch_create)."""

    def __init__(self, base_prob, Ks, Ts, cmap, params, device: int = 0, stream: Optional[int] = None,
                 schedule: int = MPPI_SCHED_AUTO):
        self.Ks = [int(k) for k in Ks]
        self.Ts = [int(t) for t in Ts]
        self.b = mppi_batch_create(make_config(base_prob, schedule=schedule), make_cost(base_prob.cost), self.Ks,
                                   self.Ts, device, 0 if stream is None else stream)
        try:
            mppi_batch_set_costmap(self.b, cmap.data, cmap.origin_x, cmap.origin_y, cmap.resolution)
            mppi_batch_set_dynamics(self.b, params)
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "b", None):
            mppi_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def iterate(self, x0):
        mppi_batch_iterate(self.b, x0)

    def controls(self, i: int):
        return mppi_batch_get_controls(self.b, i, self.Ts[i])[0]

    def costs(self, i: int):
        return mppi_batch_get_costs(self.b, i, self.Ks[i])

    def set_controls(self, i: int, U):
        mppi_batch_set_controls(self.b, i, U)

    def schedule(self):
        return mppi_batch_get_schedule(self.b)

    def synchronize(self):
        mppi_batch_synchronize(self.b)


# ---------------------------------------------------------------------------
# Convenience wrapper
# ---------------------------------------------------------------------------

def make_config(prob, precision: int = MPPI_PREC_FP32, schedule: int = MPPI_SCHED_AUTO) -> mppi_config:
    c = mppi_config()
    c.K, c.T = int(prob.K), int(prob.T)
    c.dt, c.lam = prob.dt, prob.lam
    c.gamma = prob.lam if getattr(prob, "gamma", None) is None else prob.gamma
    c.sigma2[:] = list(prob.sigma2)
    c.u_lo[:] = list(prob.u_lo)
    c.u_hi[:] = list(prob.u_hi)
    c.sg_window, c.sg_order = int(prob.sg_window), int(prob.sg_order)
    c.precision, c.schedule = precision, schedule
    c.seed = int(prob.seed)
    c.instance = int(getattr(prob, "instance", 0))
    c.explore = float(getattr(prob, "explore", 0.0))
    c.weighting = int(getattr(prob, "weighting", MPPI_WEIGHTS_IT))
    c.elite = float(getattr(prob, "elite", 0.8))
    c.k_base = int(getattr(prob, "k_base", 0))
    c.k_total = int(getattr(prob, "k_total", 0))
    return c


def make_cost(cost) -> mppi_cost:
    c = mppi_cost()
    for f, _ in mppi_cost._fields_:
        setattr(c, f, getattr(cost, f))
    return c


def current_stream() -> int:
    """The HIP stream torch uses on the current device (0 when torch/GPU is absent)."""
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover
        pass
    return 0


class Controller:
    """One MPPI controller on one GPU (owns one library context)."""

    def __init__(self, prob, cmap, params, device: int = 0, stream: Optional[int] = None,
                 precision: int = MPPI_PREC_FP32, schedule: int = MPPI_SCHED_AUTO):
        self.K, self.T, self.hidden = int(prob.K), int(prob.T), int(prob.hidden)
        self.ctx = mppi_create(make_config(prob, precision, schedule), make_cost(prob.cost), device,
                               current_stream() if stream is None else stream)
        try:
            mppi_set_costmap(self.ctx, cmap.data, cmap.origin_x, cmap.origin_y, cmap.resolution)
            self.model = int(getattr(prob, "model", 0))
            if self.model == 1:
                mppi_set_basis_dynamics(self.ctx, params)
            else:
                mppi_set_dynamics(self.ctx, self.hidden, params)
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "ctx", None):
            mppi_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_controls(self, U):
        mppi_set_controls(self.ctx, U)

    def iterate(self, x0, want_costs: bool = False):
        if want_costs:
            S = np.zeros(self.K, dtype=np.float32)
            st = mppi_iterate(self.ctx, x0, S)
            return S, st
        return None, mppi_iterate(self.ctx, x0)

    def controls(self):
        return mppi_get_controls(self.ctx, self.T)[0]

    def shift(self):
        return mppi_shift(self.ctx)[0]

    def plant_step(self, x, u):
        return mppi_plant_step(self.ctx, x, u)

    def stats(self):
        return mppi_get_stats(self.ctx, self.T)

    def noise(self, it: int):
        return mppi_get_noise(self.ctx, it, self.K, self.T)

    @property
    def iteration(self) -> int:
        return mppi_get_iteration(self.ctx)

    @iteration.setter
    def iteration(self, it: int):
        mppi_set_iteration(self.ctx, it)

    @property
    def schedule(self) -> int:
        return mppi_get_schedule(self.ctx)

    def set_dynamics(self, params):
        mppi_set_dynamics(self.ctx, self.hidden, params)
        self.model = 0

    def set_basis_dynamics(self, theta):
        mppi_set_basis_dynamics(self.ctx, theta)
        self.model = 1

    def objective(self, x0, it: int, ckpt_every: int = 10, want_costs: bool = False):
        return mppi_objective(self.ctx, x0, it, ckpt_every, self.K if want_costs else None)

    def objective_backward(self):
        return mppi_objective_backward(self.ctx, self.T)
