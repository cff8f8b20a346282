"""MI355X-native MPPI (information-theoretic model predictive control) library.

The compute lives in ``libmppi.so`` (HIP kernels for gfx950 behind the C ABI of
``include/mppi.h``); ``paper_1707_02342_amd.mppi`` is its ctypes binding.
Importing this package loads nothing; the library is loaded on first use and
its absence is an error, never a silent fallback.
"""
from .mppi import (Controller, MppiError, make_config, make_cost)  # noqa: F401

__all__ = ["Controller", "MppiError", "make_config", "make_cost"]
