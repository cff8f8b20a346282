"""Pins of the oracle's noise generator (Algorithm 1: sample E^k, eps_t ~ N(0, Sigma)).

* Philox4x32-10 against ROCm rocRAND's independent header-only engine (run live).
* The FP32 log and sin/cos of the Box-Muller transform against libm.
* The composition (counter layout, uniform construction, Box-Muller) against a
  float64 transcription of the written definition.
* Statistics of the draws: mean, variance, Kolmogorov-Smirnov, neighbour correlation.
"""
import math
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import synth

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def kat_exe(tmp_path_factory):
    src = __import__("pathlib").Path(__file__).parent / "helpers" / "rocrand_philox_kat.cpp"
    exe = tmp_path_factory.mktemp("kat") / "kat"
    try:
        subprocess.run([HIPCC, "-x", "c++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                        str(src), "-o", str(exe)], check=True, capture_output=True, timeout=300)
    except (OSError, subprocess.CalledProcessError) as e:  # pragma: no cover
        pytest.skip(f"rocRAND host build unavailable: {e}")
    return exe


def test_philox_matches_rocrand(orc, kat_exe):
    rng = np.random.default_rng(1234)
    cases = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2),
             ([1, 0, 0, 0], [0, 0]), ([0, 0, 0, 1], [0, 0]), ([99, 1919, 7, 3], [0, 0])]
    for _ in range(24):
        cases.append((list(rng.integers(0, 2**32, 4, dtype=np.uint64)),
                      list(rng.integers(0, 2**32, 2, dtype=np.uint64))))
    for ctr, key in cases:
        out = subprocess.run([str(kat_exe)] + [str(int(v)) for v in ctr + key], check=True,
                             capture_output=True, text=True).stdout.split()
        ref = np.array([int(v) for v in out], dtype=np.uint32)
        got = orc.philox4x32_10(ctr, key)
        assert np.array_equal(got, ref), (ctr, key, got, ref)


def _words(n, seed):
    rng = np.random.default_rng(seed)
    w = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    edges = np.array([0, 511, 512, 0xFFFFFFFF, 0xFFFFFE00, 0x80000000, 0x7FFFFFFF, 0x5A827999 << 1],
                     dtype=np.uint64).astype(np.uint32)
    return np.concatenate([edges, w])


def test_noise_log_against_libm(orc):
    worst = 0.0
    for w in _words(20000, 7):
        n = 2 * (int(w) >> 9) + 1
        ref = math.log(n) - 24 * math.log(2.0)
        got = float(orc.noise_log(int(w)))
        ulp = float(np.spacing(np.float32(abs(ref))))
        worst = max(worst, abs(got - ref) / ulp)
    assert worst <= 2.0, worst


def test_noise_sincos_against_libm(orc):
    worst = 0.0
    for w in _words(20000, 8):
        n = 2 * (int(w) >> 9) + 1
        a = 2.0 * math.pi * n / 2.0**24
        c, s = orc.noise_sincos(int(w))
        worst = max(worst, abs(float(c) - math.cos(a)), abs(float(s) - math.sin(a)))
    assert worst <= 2.5e-7, worst


def test_noise_composition_matches_definition(orc):
    """eps[k][t] = sqrt(Sigma) * Box-Muller(words 0,1 of Philox(ctr=(t,k,iter,instance),
    key=(seed_lo, seed_hi))), u = (2*(w>>9)+1)/2^24."""
    p = synth.with_(synth.c1_problem(), K=7, T=5, seed=0x1234567890AB, instance=3,
                    sigma2=(0.3, 0.35))
    op = orc.OracleProblem(p, synth.constant_map(0.0), synth.mlp_params(32, 0))
    it = 11
    eps = orc.noise(op, it)
    sig = np.sqrt(np.float32(p.sigma2))
    for k in range(7):
        for t in range(5):
            w = orc.philox4x32_10([t, k, it, 3], [p.seed & 0xFFFFFFFF, p.seed >> 32])
            u1 = (2 * (int(w[0]) >> 9) + 1) / 2.0**24
            u2 = (2 * (int(w[1]) >> 9) + 1) / 2.0**24
            r = math.sqrt(-2.0 * math.log(u1))
            z = (r * math.cos(2 * math.pi * u2), r * math.sin(2 * math.pi * u2))
            for i in range(2):
                assert abs(eps[k, t, i] - sig[i] * z[i]) <= 1e-6 * max(1.0, abs(z[i])), (k, t, i)


def test_noise_statistics(orc):
    p = synth.with_(synth.c1_problem(), K=32768, T=100, sigma2=(1.0, 1.0), seed=5)
    op = orc.OracleProblem(p, synth.constant_map(0.0), synth.mlp_params(32, 0))
    eps = orc.noise(op, 0).astype(np.float64)
    n = eps.shape[0] * eps.shape[1]
    for i in range(2):
        z = eps[:, :, i].ravel()
        assert abs(z.mean()) < 5.0 / math.sqrt(n)
        assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
        assert stats.kstest(z[::7], "norm").pvalue > 1e-4
    # the two channels of a pair, and neighbours in t and in k, are uncorrelated
    lim = 5.0 / math.sqrt(n)
    assert abs(np.mean(eps[:, :, 0] * eps[:, :, 1])) < lim
    assert abs(np.mean(eps[:, 1:, 0] * eps[:, :-1, 0])) < lim
    assert abs(np.mean(eps[1:, :, 1] * eps[:-1, :, 1])) < lim
    # fourth moment of a normal is 3
    assert abs(np.mean(eps[:, :, 0] ** 4) - 3.0) < 0.02


def test_noise_depends_on_every_counter_word(orc):
    base = synth.with_(synth.c1_problem(), K=4, T=4, seed=9)
    op = orc.OracleProblem(base, synth.constant_map(0.0), synth.mlp_params(32, 0))
    e0 = orc.noise(op, 0)
    assert not np.array_equal(e0, orc.noise(op, 1))                       # iteration counter
    op2 = orc.OracleProblem(synth.with_(base, instance=1), synth.constant_map(0.0), synth.mlp_params(32, 0))
    assert not np.array_equal(e0, orc.noise(op2, 0))                       # instance
    op3 = orc.OracleProblem(synth.with_(base, seed=10), synth.constant_map(0.0), synth.mlp_params(32, 0))
    assert not np.array_equal(e0, orc.noise(op3, 0))                       # seed
    assert not np.array_equal(e0[0], e0[1]) and not np.array_equal(e0[:, 0], e0[:, 1])
