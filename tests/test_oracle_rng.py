"""Pins for the oracle's random-number layer (test infrastructure).

* Philox4x32-10 against rocRAND's header-only engine, an independent library
  implementation of the same published generator.
* The uniform conversions: range and exact representability.
* Gamma variates (Marsaglia & Tsang) against scipy's log-gamma distribution
  (Kolmogorov-Smirnov) and its first two moments.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_ref.cpp")])
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(1234)
    # the reference engine addresses the low 64 counter bits in words (x4), so
    # the second counter word stays below 2^30 here
    cases = [(0, [0, 0, 0, 0]), ((1 << 64) - 1, [0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]),
             (0x0123456789ABCDEF, [1, 2, 3, 4])]
    for _ in range(3000):
        key = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        ctr = [int(v) for v in rng.integers(0, 1 << 32, size=4, dtype=np.uint64)]
        ctr[1] &= 0x3FFFFFFF
        cases.append((key, ctr))
    text = "".join("%x %x %x %x %x\n" % (k, *c) for k, c in cases)
    out = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    for (key, ctr), line in zip(cases, out):
        ref = [int(t, 16) for t in line.split()]
        got = [int(v) for v in oracle.philox4x32_10(key, ctr)]
        assert got == ref, (hex(key), ctr)


def test_uniform_conversions_exact_and_open():
    assert oracle.u23(0) == 2.0 ** -24
    assert oracle.u23(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert oracle.u52(0, 0) == 2.0 ** -53
    assert oracle.u52(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    rng = np.random.default_rng(7)
    for w in rng.integers(0, 1 << 32, size=2000, dtype=np.uint64):
        u = oracle.u23(int(w))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u          # exact in single precision
        assert (u * 2 ** 24) % 2 == 1             # odd multiple of 2^-24
        v = oracle.u52(int(w), int(w) ^ 0x5A5A5A5A)
        assert 0.0 < v < 1.0 and (v * 2 ** 53) % 2 == 1


@pytest.mark.parametrize("shape", [0.03, 0.5, 1.0, 3.7, 250.0, 1.0e6])
def test_gamma_variates_follow_gamma_law(shape):
    n = 12000
    lg = np.array([oracle.log_gamma_variate(shape, 99, i, 7, 3, oracle.ST_GAMMA) for i in range(n)])
    assert np.all(np.isfinite(lg))
    # log of a Gamma(shape, 1) variate follows scipy's loggamma(shape)
    ks = stats.kstest(lg, stats.loggamma(shape).cdf)
    assert ks.pvalue > 1e-3, ks
    m, v = stats.loggamma(shape).stats(moments="mv")
    se = math.sqrt(float(v) / n)
    assert abs(lg.mean() - float(m)) < 5 * se
    if shape >= 1.0:
        x = np.exp(lg)
        assert abs(x.mean() - shape) < 5 * math.sqrt(shape / n)
        assert abs(x.var() / shape - 1.0) < 0.1


def test_gamma_variates_are_addressed_by_counter():
    a = oracle.log_gamma_variate(2.5, 5, 10, 3, 4, oracle.ST_GAMMA)
    assert a == oracle.log_gamma_variate(2.5, 5, 10, 3, 4, oracle.ST_GAMMA)
    others = [oracle.log_gamma_variate(2.5, 6, 10, 3, 4, oracle.ST_GAMMA),
              oracle.log_gamma_variate(2.5, 5, 11, 3, 4, oracle.ST_GAMMA),
              oracle.log_gamma_variate(2.5, 5, 10, 4, 4, oracle.ST_GAMMA),
              oracle.log_gamma_variate(2.5, 5, 10, 3, 5, oracle.ST_GAMMA),
              oracle.log_gamma_variate(2.5, 5, 10, 3, 4, oracle.ST_PI)]
    assert all(o != a for o in others)
