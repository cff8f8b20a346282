"""Build libmppi.so (HIP, gfx950) in-tree with hipcc.

All device code is compiled for gfx950 only, with -ffp-contract=off (fused
multiply-adds only where the source writes them) and packed-FP32 instructions
disabled.  The library is placed next to this file so that it travels with the
source tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libmppi.so"

SOURCES = ["mppi_runtime.hip", "kernels_lane.hip", "kernels_wave.hip", "kernels_wave_split.hip", "kernels_wide.hip", "kernels_quad.hip",
           "kernels_adjoint.hip", "kernels_update.hip", "kernels_cem.hip"]

HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> Path:
    srcs = [str(CSRC / s) for s in SOURCES]
    tmp = LIB.with_name(LIB.name + ".tmp")
    cmd = [hipcc(), *HIPFLAGS, "-I", str(ROOT / "include"), "-I", str(CSRC), *srcs, "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmppi.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
