"""Test mode of the oracle: built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, host code only), and the CPU test suite run against that build.

    python oracle/sanitize.py [extra pytest arguments]

The instrumented library is oracle/liboracle_asan.so; the suite loads it in place of
liboracle.so through MPPI_ORACLE_LIB, with the ASan runtime preloaded into the Python
process (leak detection off: the interpreter itself keeps allocations until exit).  Any
sanitizer report ends the run with a non-zero status.
"""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402

SAN_LIB = HERE / "liboracle_asan.so"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build() -> Path:
    flags = [f for f in oracle.CXXFLAGS if f != "-O2"] + ["-O1"] + SAN_FLAGS
    subprocess.run(["g++", *flags, str(oracle.SRC), "-o", str(SAN_LIB)], check=True)
    return SAN_LIB


def main(argv) -> int:
    build()
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    env = dict(os.environ)
    env.update({"MPPI_ORACLE_LIB": str(SAN_LIB), "LD_PRELOAD": asan,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    cmd = [sys.executable, "-m", "pytest", str(ROOT / "tests"), "-m", "not gpu", "-x", "-q", *argv]
    print("sanitized oracle:", SAN_LIB, flush=True)
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
