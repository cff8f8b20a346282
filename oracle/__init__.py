"""ctypes wrapper of the CPU oracle (oracle/oracle.cpp).

TEST INFRASTRUCTURE ONLY: the oracle is what the GPU library is checked
against.  Only the tests, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It never imports the GPU
library, and the GPU library never imports it.

Inputs are accepted duck-typed (any object with the problem's fields, any map
object with ``data/origin_x/origin_y/resolution``) so that this package does not
depend on the input generators either.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "oracle.cpp"
PLAIN_LIB = HERE / "liboracle.so"
# the library loaded: MPPI_ORACLE_LIB names another build of the same source (the
# sanitizer test mode, oracle/sanitize.py); by default the plain build
LIB = Path(os.environ.get("MPPI_ORACLE_LIB", PLAIN_LIB))

OK, E_INVAL, E_NONFINITE = 0, 1, 5
WEIGHTS_IT, WEIGHTS_CEM = 0, 1
MODEL_NET, MODEL_BASIS = 0, 1

CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-pthread", "-Wall", "-Wextra"]


def build(force: bool = True) -> Path:
    """Compile the oracle with g++ (plain C++17, no contraction, IEEE div/sqrt)."""
    if force or not PLAIN_LIB.exists():
        tmp = PLAIN_LIB.with_suffix(".so.tmp")
        subprocess.run(["g++", *CXXFLAGS, str(SRC), "-o", str(tmp)], check=True)
        os.replace(tmp, PLAIN_LIB)
    return PLAIN_LIB


class Problem(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("T", C.c_int32), ("hidden", C.c_int32),
        ("dt", C.c_float), ("lam", C.c_float), ("gamma", C.c_float),
        ("sigma2", C.c_float * 2), ("u_lo", C.c_float * 2), ("u_hi", C.c_float * 2),
        ("sg_window", C.c_int32), ("sg_order", C.c_int32),
        ("w_map", C.c_float), ("w_speed", C.c_float), ("w_slip", C.c_float), ("v_des", C.c_float),
        ("crash_cost", C.c_float), ("crash_decay", C.c_float), ("map_thresh", C.c_float),
        ("slip_cost", C.c_float), ("slip_thresh", C.c_float),
        ("H", C.c_int32), ("W", C.c_int32),
        ("origin_x", C.c_float), ("origin_y", C.c_float), ("resolution", C.c_float),
        ("map", C.POINTER(C.c_float)), ("params", C.POINTER(C.c_float)),
        ("seed", C.c_uint64), ("instance", C.c_uint32), ("explore", C.c_float),
        ("weighting", C.c_int32), ("elite", C.c_float), ("model", C.c_int32), ("nthreads", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB.exists():
            if LIB != PLAIN_LIB:
                raise ImportError(f"{LIB} (MPPI_ORACLE_LIB) does not exist")
            build(force=True)
        L = C.CDLL(str(LIB))
        fp = C.POINTER(C.c_float)
        dp = C.POINTER(C.c_double)
        u32p = C.POINTER(C.c_uint32)
        pp = C.POINTER(Problem)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_noise_log.argtypes = [C.c_uint32]
        L.orc_noise_log.restype = C.c_float
        L.orc_noise_sincos.argtypes = [C.c_uint32, fp, fp]
        L.orc_noise.argtypes = [pp, C.c_uint32, fp]
        L.orc_rollout_f64.argtypes = [pp, fp, fp, fp, dp, dp]
        L.orc_rollout_f32.argtypes = [pp, fp, fp, fp, fp, fp]
        L.orc_weights.argtypes = [C.c_int, dp, C.c_double, dp, dp, dp]
        L.orc_cem_zeta.argtypes = [C.c_int, C.c_float]
        L.orc_cem_zeta.restype = C.c_int
        L.orc_weights_cem.argtypes = [C.c_int, dp, C.c_int, dp, dp, dp]
        L.orc_weights_cem.restype = C.c_int
        L.orc_sgf_matrix.argtypes = [C.c_int, C.c_int, C.c_int, dp]
        L.orc_iterate.argtypes = [pp, fp, fp, C.c_uint32, fp, dp, dp, dp, dp, dp]
        L.orc_shift.argtypes = [C.c_int, dp, dp, dp]
        L.orc_plant_step.argtypes = [pp, dp, dp, dp]
        L.orc_objective.argtypes = [pp, fp, dp, dp, C.c_uint32, dp, dp]
        L.orc_objective_grad.argtypes = [pp, fp, dp, dp, C.c_uint32, dp, dp, dp]
        L.orc_toy_iterate.argtypes = [C.c_double, C.c_double, C.c_double, C.c_float, C.c_float,
                                      C.c_double, C.c_int, C.c_int, dp, C.c_uint64, C.c_uint32,
                                      C.c_double, dp]
        L.orc_threshold_margins.argtypes = [pp, fp, fp, fp, dp]
        L.orc_threshold_margins.restype = C.c_int
        i32p = C.POINTER(C.c_int32)
        L.orc_threshold_events.argtypes = [pp, fp, fp, fp, C.c_double, C.c_int32, i32p, i32p, i32p, dp, i32p]
        L.orc_threshold_events.restype = C.c_int
        L.orc_mlp_forward.argtypes = [pp, dp, dp]
        L.orc_basis_phi.argtypes = [dp, dp, dp]
        L.orc_costmap.argtypes = [pp, C.c_double, C.c_double, dp]
        L.orc_costmap.restype = C.c_double
        L.orc_state_cost.argtypes = [pp, dp, C.c_int, dp]
        L.orc_state_cost.restype = C.c_double
        for name in ("orc_mlp_forward", "orc_rollout_f64", "orc_rollout_f32", "orc_weights", "orc_iterate",
                     "orc_objective", "orc_objective_grad", "orc_toy_iterate"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class OracleProblem:
    """Holds a populated ``Problem`` struct plus the arrays it points to."""

    def __init__(self, prob, cmap, params, nthreads: int = 0, K: int | None = None,
                 T: int | None = None):
        cost = prob.cost
        self.map = _f32(cmap.data)
        self.params = _f32(params)
        s = Problem()
        s.K = int(prob.K if K is None else K)
        s.T = int(prob.T if T is None else T)
        s.hidden = int(prob.hidden)
        s.dt = prob.dt
        s.lam = prob.lam
        s.gamma = prob.lam if getattr(prob, "gamma", None) is None else prob.gamma
        s.sigma2[:] = list(prob.sigma2)
        s.u_lo[:] = list(prob.u_lo)
        s.u_hi[:] = list(prob.u_hi)
        s.sg_window = int(prob.sg_window)
        s.sg_order = int(prob.sg_order)
        for f in ("w_map", "w_speed", "w_slip", "v_des", "crash_cost", "crash_decay",
                  "map_thresh", "slip_cost", "slip_thresh"):
            setattr(s, f, getattr(cost, f))
        s.H, s.W = int(self.map.shape[0]), int(self.map.shape[1])
        s.origin_x, s.origin_y, s.resolution = cmap.origin_x, cmap.origin_y, cmap.resolution
        s.map = _ptr(self.map, C.c_float)
        s.params = _ptr(self.params, C.c_float)
        s.seed = int(prob.seed)
        s.instance = int(getattr(prob, "instance", 0))
        s.explore = float(getattr(prob, "explore", 0.0))
        s.weighting = int(getattr(prob, "weighting", WEIGHTS_IT))
        s.elite = float(getattr(prob, "elite", 0.8))
        s.model = int(getattr(prob, "model", MODEL_NET))
        s.nthreads = int(nthreads or min(16, os.cpu_count() or 1))
        self.s = s

    @property
    def K(self):
        return self.s.K

    @property
    def T(self):
        return self.s.T

    def ref(self):
        return C.byref(self.s)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def noise_log(w: int) -> np.float32:
    return np.float32(lib().orc_noise_log(int(w)))


def noise_sincos(w: int):
    c, s = C.c_float(), C.c_float()
    lib().orc_noise_sincos(int(w), C.byref(c), C.byref(s))
    return np.float32(c.value), np.float32(s.value)


def noise(op: OracleProblem, it: int = 0) -> np.ndarray:
    eps = np.zeros((op.K, op.T, 2), dtype=np.float32)
    lib().orc_noise(op.ref(), it, _ptr(eps, C.c_float))
    return eps


def rollout(op: OracleProblem, x0, U, eps, precision: str = "f64", traj: bool = False):
    x0 = _f32(x0)
    U = _f32(U)
    eps = _f32(eps)
    K, T = op.K, op.T
    if precision == "f64":
        S = np.zeros(K, dtype=np.float64)
        tr = np.zeros((K, T + 1, 7), dtype=np.float64) if traj else None
        st = lib().orc_rollout_f64(op.ref(), _ptr(x0, C.c_float), _ptr(U, C.c_float), _ptr(eps, C.c_float),
                                   _ptr(S, C.c_double), _ptr(tr, C.c_double) if traj else None)
    else:
        S = np.zeros(K, dtype=np.float32)
        tr = np.zeros((K, T + 1, 7), dtype=np.float32) if traj else None
        st = lib().orc_rollout_f32(op.ref(), _ptr(x0, C.c_float), _ptr(U, C.c_float), _ptr(eps, C.c_float),
                                   _ptr(S, C.c_float), _ptr(tr, C.c_float) if traj else None)
    if st != OK:
        raise ValueError(f"oracle rollout status {st}")
    return (S, tr) if traj else S


def weights(S, lam: float):
    S = _f64(S)
    w = np.zeros_like(S)
    rho, eta = C.c_double(), C.c_double()
    st = lib().orc_weights(S.size, _ptr(S, C.c_double), float(lam), _ptr(w, C.c_double),
                           C.byref(rho), C.byref(eta))
    return st, w, rho.value, eta.value


def cem_zeta(K: int, elite: float) -> int:
    return int(lib().orc_cem_zeta(int(K), float(elite)))


def weights_cem(S, zeta: int):
    """Algorithm 3: (status, w, largest elite cost, elite count)."""
    S = _f64(S)
    w = np.zeros_like(S)
    z, n = C.c_double(), C.c_double()
    st = lib().orc_weights_cem(S.size, _ptr(S, C.c_double), int(zeta), _ptr(w, C.c_double),
                               C.byref(z), C.byref(n))
    if st == E_INVAL:
        raise ValueError("oracle: invalid CEM arguments")
    return st, w, z.value, int(n.value)


def sgf_matrix(T: int, window: int, order: int) -> np.ndarray:
    M = np.zeros((T, T), dtype=np.float64)
    lib().orc_sgf_matrix(T, window, order, _ptr(M, C.c_double))
    return M


class IterResult:
    def __init__(self, status, U, S, w, delta, rho, eta):
        self.status, self.U, self.S, self.w, self.delta, self.rho, self.eta = status, U, S, w, delta, rho, eta


def iterate(op: OracleProblem, x0, U, it: int = 0, eps=None) -> IterResult:
    x0 = _f32(x0)
    U = _f32(U)
    K, T = op.K, op.T
    Uo = np.zeros((T, 2), dtype=np.float64)
    S = np.zeros(K)
    w = np.zeros(K)
    d = np.zeros((T, 2))
    re = np.zeros(2)
    e = _f32(eps) if eps is not None else None
    st = lib().orc_iterate(op.ref(), _ptr(x0, C.c_float), _ptr(U, C.c_float), it,
                           _ptr(e, C.c_float) if e is not None else None,
                           _ptr(Uo, C.c_double), _ptr(S, C.c_double), _ptr(w, C.c_double),
                           _ptr(d, C.c_double), _ptr(re, C.c_double))
    if st == E_INVAL:
        raise ValueError("oracle: invalid problem")
    return IterResult(st, Uo, S, w, d, re[0], re[1])


def shift(U):
    U = _f64(U)
    T = U.shape[0]
    Uo = np.zeros_like(U)
    u0 = np.zeros(2)
    lib().orc_shift(T, _ptr(U, C.c_double), _ptr(Uo, C.c_double), _ptr(u0, C.c_double))
    return Uo, u0


def plant_step(op: OracleProblem, x, u) -> np.ndarray:
    x = _f64(x)
    u = _f64(u)
    out = np.zeros(7)
    lib().orc_plant_step(op.ref(), _ptr(x, C.c_double), _ptr(u, C.c_double), _ptr(out, C.c_double))
    return out


def objective(op: OracleProblem, x0, U, params=None, it: int = 0):
    x0 = _f32(x0)
    U = _f64(U)
    P = _f64(params) if params is not None else None
    J = C.c_double()
    S = np.zeros(op.K)
    st = lib().orc_objective(op.ref(), _ptr(x0, C.c_float), _ptr(U, C.c_double),
                             _ptr(P, C.c_double) if P is not None else None, it, C.byref(J),
                             _ptr(S, C.c_double))
    if st != OK:
        raise ValueError(f"oracle objective status {st}")
    return J.value, S


def objective_grad(op: OracleProblem, x0, U, params=None, it: int = 0):
    x0 = _f32(x0)
    U = _f64(U)
    P = _f64(params) if params is not None else None
    J = C.c_double()
    gU = np.zeros((op.T, 2))
    h = op.s.hidden
    gth = np.zeros(6 * h + h + h * h + h + 4 * h + 4)
    st = lib().orc_objective_grad(op.ref(), _ptr(x0, C.c_float), _ptr(U, C.c_double),
                                  _ptr(P, C.c_double) if P is not None else None, it, C.byref(J),
                                  _ptr(gU, C.c_double), _ptr(gth, C.c_double))
    if st != OK:
        raise ValueError(f"oracle objective_grad status {st}")
    return J.value, gU, gth


def toy_iterate(a, b, q, lam, sigma2, x0, U, K, seed=0, it=0, ctrl_scale=1.0):
    U = _f64(U)
    T = U.size
    Uo = np.zeros(T)
    st = lib().orc_toy_iterate(a, b, q, lam, sigma2, x0, T, K, _ptr(U, C.c_double), seed, it,
                               float(ctrl_scale), _ptr(Uo, C.c_double))
    if st != OK:
        raise ValueError(f"oracle toy status {st}")
    return Uo


def mlp_forward(op: OracleProblem, inp) -> np.ndarray:
    x = _f64(inp)
    out = np.zeros(4)
    st = lib().orc_mlp_forward(op.ref(), _ptr(x, C.c_double), _ptr(out, C.c_double))
    if st != OK:
        raise ValueError("oracle mlp status")
    return out


def basis_phi(xd, u) -> np.ndarray:
    """The 25 basis functions at x_d = (roll, v_x, v_y, heading rate), u = (steer, throttle)."""
    x = _f64(xd)
    uu = _f64(u)
    out = np.zeros(25)
    lib().orc_basis_phi(_ptr(x, C.c_double), _ptr(uu, C.c_double), _ptr(out, C.c_double))
    return out


def costmap(op: OracleProblem, px: float, py: float):
    g = np.zeros(2)
    h = lib().orc_costmap(op.ref(), float(px), float(py), _ptr(g, C.c_double))
    return h, g


def state_cost(op: OracleProblem, x, t: int):
    x = _f64(x)
    g = np.zeros(7)
    c = lib().orc_state_cost(op.ref(), _ptr(x, C.c_double), int(t), _ptr(g, C.c_double))
    return c, g


def threshold_margins(op: OracleProblem, x0, U, eps) -> np.ndarray:
    x0 = _f32(x0)
    U = _f32(U)
    eps = _f32(eps)
    m = np.zeros(op.K)
    st = lib().orc_threshold_margins(op.ref(), _ptr(x0, C.c_float), _ptr(U, C.c_float),
                                     _ptr(eps, C.c_float), _ptr(m, C.c_double))
    if st != OK:
        raise ValueError("oracle margins status")
    return m


class ThresholdEvents:
    """The impulse terms a sample's FP64 trajectory decides within `window` of their
    threshold (oracle.cpp, orc_threshold_events): per sample k, the lists t[k], kind[k]
    (0 crash, 1 slip), value[k] (the term's size) and on[k] (whether the oracle's
    trajectory takes it)."""

    def __init__(self, n, t, kind, value, on):
        self.n, self.t, self.kind, self.value, self.on = n, t, kind, value, on

    def taken(self) -> np.ndarray:
        """Per sample, the sum of the listed terms the oracle takes."""
        return np.array([float(np.sum(v[o.astype(bool)])) for v, o in zip(self.value, self.on)])


def threshold_events(op: OracleProblem, x0, U, eps, window: float = 1e-4, cap: int = 64) -> ThresholdEvents:
    x0 = _f32(x0)
    U = _f32(U)
    eps = _f32(eps)
    K = op.K
    n = np.zeros(K, np.int32)
    t = np.zeros((K, cap), np.int32)
    kind = np.zeros((K, cap), np.int32)
    val = np.zeros((K, cap), np.float64)
    on = np.zeros((K, cap), np.int32)
    st = lib().orc_threshold_events(op.ref(), _ptr(x0, C.c_float), _ptr(U, C.c_float), _ptr(eps, C.c_float),
                                    float(window), int(cap), _ptr(n, C.c_int32), _ptr(t, C.c_int32),
                                    _ptr(kind, C.c_int32), _ptr(val, C.c_double), _ptr(on, C.c_int32))
    if st != OK:
        raise ValueError("oracle threshold events status")
    if n.max(initial=0) > cap:
        raise ValueError(f"a sample has {n.max()} near-threshold terms, more than cap={cap}")
    return ThresholdEvents(n, [t[k, :n[k]] for k in range(K)], [kind[k, :n[k]] for k in range(K)],
                           [val[k, :n[k]] for k in range(K)], [on[k, :n[k]] for k in range(K)])
