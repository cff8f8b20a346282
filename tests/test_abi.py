"""Host-side checks of the C-ABI library (no GPU needed): it loads, it exports every
entry point include/mppi.h declares, the binding names match, and argument validation
rejects bad input before any device work.  No compute call is made here."""
import ctypes as C
import re
from pathlib import Path

import numpy as np
import pytest

import synth

ROOT = Path(__file__).resolve().parent.parent


@pytest.fixture(scope="module")
def M():
    from paper_1707_02342_amd import mppi
    if not mppi.LIB_PATH.exists():
        from paper_1707_02342_amd import build
        build.build()
    mppi.lib()
    return mppi


def header_functions():
    text = (ROOT / "include" / "mppi.h").read_text()
    return sorted(set(re.findall(r"\b(mppi_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(M):
    names = header_functions()
    assert len(names) >= 15
    L = M.lib()
    for n in names:
        assert hasattr(L, n), f"libmppi.so does not export {n}"
    assert sorted(M.EXPORTED) == names
    for n in names:
        assert callable(getattr(M, n)), f"binding lacks {n}"


def test_struct_layout_matches_header(M):
    # int32 K, T; float dt, lambda, gamma, sigma2[2], u_lo[2], u_hi[2]; int32 sg_window, sg_order,
    # precision, schedule; uint64 seed; uint32 instance; float explore; int32 weighting;
    # float elite; uint32 k_base; int32 k_total -> 15*4 + pad 4 + 8 + 6*4 = 96
    assert C.sizeof(M.mppi_config) == 96
    assert M.mppi_config.seed.offset == 64
    assert M.mppi_config.explore.offset == 76
    assert M.mppi_config.weighting.offset == 80
    assert M.mppi_config.elite.offset == 84
    assert M.mppi_config.k_base.offset == 88
    assert M.mppi_config.k_total.offset == 92
    assert C.sizeof(M.mppi_cost) == 36


def _cfg(M, **kw):
    c = M.make_config(synth.c1_problem())
    for k, v in kw.items():
        if k in ("sigma2", "u_lo", "u_hi"):
            getattr(c, k)[:] = v
        else:
            setattr(c, k, v)
    return c


@pytest.mark.parametrize("field,value", [
    ("K", 0), ("K", -3), ("K", (1 << 22) + 1), ("T", 0), ("T", 257), ("dt", 0.0), ("dt", float("nan")),
    ("lam", 0.0), ("lam", -1.0), ("lam", float("inf")), ("gamma", float("nan")),
    ("sigma2", (0.0, 0.3)), ("sigma2", (0.3, -1.0)), ("sigma2", (float("inf"), 0.3)),
    ("u_lo", (1.5, -1.0)), ("sg_window", 2), ("sg_window", 0), ("sg_window", 31),
    ("sg_order", 1), ("precision", 7), ("schedule", 9),
    ("k_base", 5), ("k_total", 100), ("k_total", -1), ("k_total", (1 << 30) + 1),
])
def test_create_rejects_invalid_config(M, field, value):
    cfg = _cfg(M, **{field: value})
    out = C.c_void_p()
    st = M.lib().mppi_create(C.byref(cfg), C.byref(M.make_cost(synth.c1_problem().cost)), 0, None, C.byref(out))
    assert st == M.MPPI_E_INVAL
    assert out.value is None
    assert M.mppi_last_error(None) != ""


def test_create_rejects_null_and_bad_cost(M):
    out = C.c_void_p()
    cfg = _cfg(M)
    assert M.lib().mppi_create(None, None, 0, None, C.byref(out)) == M.MPPI_E_INVAL
    cost = M.make_cost(synth.c1_problem().cost)
    cost.w_map = float("nan")
    assert M.lib().mppi_create(C.byref(cfg), C.byref(cost), 0, None, C.byref(out)) == M.MPPI_E_INVAL
    assert M.lib().mppi_create(C.byref(cfg), C.byref(M.make_cost(synth.c1_problem().cost)), 0, None, None) \
        == M.MPPI_E_INVAL


def test_null_context_calls_are_rejected(M):
    L = M.lib()
    buf = np.zeros(16, np.float32)
    p = buf.ctypes.data_as(C.POINTER(C.c_float))
    assert L.mppi_iterate(None, p, None) == M.MPPI_E_INVAL
    assert L.mppi_get_controls(None, p) == M.MPPI_E_INVAL
    assert L.mppi_shift(None, p) == M.MPPI_E_INVAL
    assert L.mppi_set_controls(None, p) == M.MPPI_E_INVAL
    L.mppi_destroy(None)            # NULL-safe


def test_valid_config_without_gpu_reports_device_error(M):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    out = C.c_void_p()
    cfg = _cfg(M)
    st = M.lib().mppi_create(C.byref(cfg), C.byref(M.make_cost(synth.c1_problem().cost)), 0, None, C.byref(out))
    assert st == M.MPPI_E_DEVICE
    assert "device" in M.mppi_last_error(None).lower()


def test_binding_fails_loudly_without_library(M, monkeypatch, tmp_path):
    monkeypatch.setattr(M, "_lib", None)
    monkeypatch.setattr(M, "LIB_PATH", tmp_path / "missing.so")
    with pytest.raises(ImportError):
        M.lib()


@pytest.mark.parametrize("case", ["K", "window", "cem", "null_map", "null_U", "dims", "wave_h64", "bad_map"])
def test_iterate_noalloc_rejects_before_device_work(M, case):
    """The allocation-free entry point validates everything it can before touching a
    device: its size limits, Algorithm 3, NULL buffers and the network shape."""
    prob = synth.c1_problem()
    cfg = M.make_config(prob)
    cost = M.make_cost(prob.cost)
    dims = (C.c_int32 * 4)(6, 32, 32, 4)
    ptr = C.c_void_p(0x1000)            # never dereferenced: every case fails validation
    args = dict(map_dev=ptr, H=256, W=256, params=ptr, x0=ptr, U=ptr)
    if case == "K":
        cfg.K = 16385
    elif case == "window":
        cfg.T, cfg.sg_window, cfg.sg_order = 64, 33, 2
    elif case == "cem":
        cfg.weighting = M.MPPI_WEIGHTS_CEM
    elif case == "null_map":
        args["map_dev"] = None
    elif case == "null_U":
        args["U"] = None
    elif case == "dims":
        dims = (C.c_int32 * 4)(6, 48, 48, 4)
    elif case == "wave_h64":
        cfg.schedule = M.MPPI_SCHED_WAVE
        dims = (C.c_int32 * 4)(6, 64, 64, 4)
    elif case == "bad_map":
        args["H"] = 1
    st = M.lib().mppi_iterate_noalloc(C.byref(cfg), C.byref(cost), 0, None, args["map_dev"], args["H"], 256,
                                      0.0, 0.0, 0.1, dims, args["params"], args["x0"], 0, args["U"], None, None)
    assert st == M.MPPI_E_INVAL
    assert M.mppi_last_error(None) != ""


def test_shard_config_rules(M):
    """A shard must fit its iteration (k_base + K <= k_total), and Algorithm 3 and the
    batched form are unsharded; all rejected before any device work."""
    cost = M.make_cost(synth.c1_problem().cost)
    out = C.c_void_p()
    cfg = _cfg(M, k_base=200, k_total=400)          # K = 256: 200 + 256 > 400
    assert M.lib().mppi_create(C.byref(cfg), C.byref(cost), 0, None, C.byref(out)) == M.MPPI_E_INVAL
    cfg = _cfg(M, k_base=0, k_total=512, weighting=M.MPPI_WEIGHTS_CEM)
    assert M.lib().mppi_create(C.byref(cfg), C.byref(cost), 0, None, C.byref(out)) == M.MPPI_E_INVAL
    assert "Algorithm 3" in M.mppi_last_error(None)
    cfg = _cfg(M, k_base=0, k_total=512)
    Ks = (C.c_int32 * 1)(256)
    Ts = (C.c_int32 * 1)(30)
    assert M.lib().mppi_batch_create(C.byref(cfg), C.byref(cost), 1, Ks, Ts, 0, None, C.byref(out)) \
        == M.MPPI_E_INVAL
    assert "unsharded" in M.mppi_last_error(None)
