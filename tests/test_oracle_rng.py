"""Pins of the reference's random-number layer.

* Philox4x32-10 against rocRAND's implementation of the same block function (an
  independent third-party implementation, compiled here for the host).
* u24 / u53 exactness and range, from their definitions in exact rational arithmetic.
* Box-Muller normals against N(0,1) (Kolmogorov-Smirnov).
"""
import os
import shutil
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "probe")
    subprocess.run([hipcc, "--offload-host-only", "-O1", os.path.join(HERE, "rocrand_philox_probe.cpp"), "-o",
                    exe], check=True, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_probe):
    rng = np.random.default_rng(123)
    rows = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = 2**32 - 1
    # counters shaped like the ones the sampler uses
    rows[2] = [5, 17, (3 << 16) | 42, (1 << 24) | (2 << 16) | 1, 7, 0]
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    assert ref.shape == (len(rows), 4)
    for r, want in zip(rows, ref):
        got = O.philox(r[:4], r[4:6])
        assert np.array_equal(got.astype(np.uint64), want), (r, got, want)


def test_u24_exact_and_open_interval():
    rng = np.random.default_rng(1)
    xs = list(rng.integers(0, 2**32, size=5000)) + [0, 1, 511, 512, 2**32 - 1]
    for x in xs:
        x = int(x)
        u = O.u24(x)
        want = Fraction(2 * (x >> 9) + 1, 2**24)
        assert Fraction(u) == want
        assert 0 < u < 1
        assert np.float32(u) == u  # representable in FP32


def test_u53_exact_and_open_interval():
    rng = np.random.default_rng(2)
    for _ in range(5000):
        lo, hi = (int(v) for v in rng.integers(0, 2**32, size=2))
        u = O.u53(lo, hi)
        x = (hi << 32) | lo
        assert Fraction(u) == Fraction(2 * (x >> 12) + 1, 2**53)
        assert 0 < u < 1
    assert O.u53(0, 0) == 2.0**-53
    assert O.u53(2**32 - 1, 2**32 - 1) == 1 - 2.0**-53


def test_box_muller_normal_ks():
    z = np.array([O.normal_call(99, [i, 0, 1 << 16, (4 << 24) | 0]) for i in range(20000)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 4 / np.sqrt(len(z))
    assert abs(z.var() - 1) < 0.05
