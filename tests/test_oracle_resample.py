"""Pins of the integer systematic resampling (Sec. IV-B, Eq. cdf and ncopies, Alg. 1).

The reference's ancestors are compared bit-for-bit with an exact-rational
implementation written directly from the paper's equations: cdf^i = N sum_{j<=i} w_j,
ncopies^i = ceil(cdf^i - u) - ceil(cdf^{i-1} - u) (the paper's index shifted so that
it refers to cdf^0 = 0 ... cdf^N), followed by the sequential redistribution of
Alg. 1. The weights are w_j = q_j / Q and the uniform is u = floor(x64 Q / 2^64) / Q in
[0, 1), x64 being the 64-bit random word.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def paper_systematic(q, x64):
    N = len(q)
    Q = int(sum(int(v) for v in q))
    U = int(x64) * Q >> 64
    u = Fraction(U, Q)
    cdf = [Fraction(0)]
    acc = 0
    for v in q:
        acc += int(v)
        cdf.append(Fraction(N * acc, Q))
    ncopies = [math.ceil(cdf[i] - u) - math.ceil(cdf[i - 1] - u) for i in range(1, N + 1)]
    # Alg. 1 (sequential redistribution): copy sample j ncopies[j] times
    anc = []
    for j in range(N):
        anc.extend([j] * ncopies[j])
    return np.array(anc, dtype=np.int32), np.array(ncopies)


def random_q(rng, n, kind):
    if kind == "uniform":
        w = rng.random(n)
    elif kind == "peaked":
        w = np.exp(rng.normal(0, 4, n))
    elif kind == "sparse":
        w = np.where(rng.random(n) < 0.1, rng.random(n), 0.0)
        w[rng.integers(n)] = 1.0
    else:
        w = np.ones(n)
    w = w / w.max()
    return np.floor(w * 2.0**32).astype(np.uint64)


@pytest.mark.parametrize("kind", ["uniform", "peaked", "sparse", "equal"])
@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 500, 1024, 4099])
def test_ancestors_match_paper_equations(kind, n):
    rng = np.random.default_rng(n * 31 + len(kind))
    for rep in range(6):
        q = random_q(rng, n, kind)
        x64 = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        if rep == 0:
            x64 = 0
        if rep == 1:
            x64 = 2**64 - 1
        want, ncopies = paper_systematic(q, x64)
        got = O.resample_ancestors(q, x64)
        assert np.array_equal(got, want)
        # Eq. ncopies_definition: 0 <= ncopies <= N and sum ncopies = N
        assert ncopies.sum() == n and ncopies.min() >= 0 and ncopies.max() <= n
        # systematic resampling: ncopies_j is floor(N w_j) or floor(N w_j) + 1
        Q = int(q.astype(object).sum())
        for j in range(n):
            lo = (n * int(q[j])) // Q
            assert lo <= ncopies[j] <= lo + 1


def test_equal_weights_give_identity():
    q = np.full(100, 2**32, dtype=np.uint64)
    for x64 in [0, 12345, 2**64 - 1]:
        assert np.array_equal(O.resample_ancestors(q, x64), np.arange(100))


def test_one_hot():
    q = np.zeros(50, dtype=np.uint64)
    q[17] = 2**32
    assert np.all(O.resample_ancestors(q, 987654321) == 17)


@pytest.mark.parametrize("n", [2, 10, 512, 2048, 16384])
def test_trigger_is_exact_ess_half(n):
    rng = np.random.default_rng(n)
    for rep in range(40):
        w = np.exp(rng.normal(0, rng.uniform(0.1, 3.0), n))
        q = np.floor(w / w.max() * 2.0**32).astype(np.uint64)
        qs = [int(v) >> 8 for v in q]
        ess = Fraction(sum(qs) ** 2, sum(v * v for v in qs))
        assert O.resample_trigger(q) == (ess < Fraction(n, 2))
    # boundary: ESS exactly n/2 must not trigger (strict <)
    if n % 2 == 0:
        q = np.zeros(n, dtype=np.uint64)
        q[: n // 2] = 2**32
        assert not O.resample_trigger(q)
        q[n // 2] = 2**31  # ESS slightly above n/2 -> still no resampling
        assert not O.resample_trigger(q)
    q = np.zeros(n, dtype=np.uint64)
    q[0] = 2**32
    assert O.resample_trigger(q) == (n > 2)


def test_multinomial_ancestors_have_the_weight_marginals():
    """Multinomial resampling (the particle filter's scheme in Sec. II): every slot's
    ancestor is j with probability q_j / Q, over independent streams (chi-square)."""
    from scipy import stats
    q = np.array([5, 1, 0, 9, 3, 2, 12], dtype=np.uint64) << np.uint64(20)
    p = q.astype(float) / q.sum()
    n = q.size
    counts = np.zeros(n)
    for filt in range(20000):
        anc = O.resample_multinomial(q, 7, filt, 3)
        counts += np.bincount(anc, minlength=n)
    assert counts[2] == 0  # zero weight, never chosen
    nz = p > 0
    chi2 = (((counts - counts.sum() * p) ** 2)[nz] / (counts.sum() * p[nz])).sum()
    assert stats.chi2.sf(chi2, nz.sum() - 1) > 1e-3


def test_multinomial_copies_vary_like_a_multinomial():
    """The number of copies of particle j is Binomial(n, q_j / Q): its variance
    n p (1 - p) is far above systematic resampling's (< 1/4)."""
    rng = np.random.default_rng(4)
    n = 64
    q = (rng.uniform(0.2, 1.0, n) * 2**32).astype(np.uint64)
    p = q.astype(float) / q.astype(float).sum()
    R = 4000
    copies = np.array([np.bincount(O.resample_multinomial(q, 11, f, 5), minlength=n) for f in range(R)])
    var = copies.var(0)
    expect = n * p * (1 - p)
    assert np.all(np.abs(copies.mean(0) - n * p) < 5 * np.sqrt(expect / R))
    assert np.mean(var / expect) == pytest.approx(1.0, abs=0.06)
    sys_copies = np.array([np.bincount(O.resample_ancestors(q, (f * 0x9E3779B97F4A7C15) % 2**64), minlength=n)
                           for f in range(200)])
    assert sys_copies.var(0).max() <= 0.25 + 1e-12


def test_multinomial_ancestor_is_the_first_scan_entry_above_its_uniform():
    """Brute force on a tiny case: the ancestor of slot m is min{j : C_j > U_m}."""
    q = np.array([3, 0, 7, 1, 4], dtype=np.uint64) << np.uint64(28)
    C = np.cumsum(q.astype(object))
    Q = int(C[-1])
    for filt in range(50):
        anc = O.resample_multinomial(q, 13, filt, 9)
        for m in range(q.size):
            w = O.philox([m >> 1, filt, 9, (2 << 24) | (1 << 16)], [13, 0])
            x64 = int(w[2]) | (int(w[3]) << 32) if m & 1 else int(w[0]) | (int(w[1]) << 32)
            U = (x64 * Q) >> 64
            assert anc[m] == next(j for j in range(q.size) if C[j] > U)
