"""Pins of the reference's binomial sampler and observation densities.

The binomial sampler (inversion for n*p < 10, BTRS otherwise, in FP32 and FP64) is
checked against the exact binomial pmf (scipy.stats.binom) with a chi-square test on
200k draws per (n, p) cell, plus exact edge cases. The observation log-pmfs are
checked against scipy.stats.poisson / nbinom.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O

CELLS = [
    (1, 0.3), (5, 0.5), (7, 0.02), (30, 0.2), (30, 0.5), (30, 0.9), (100, 0.099), (100, 0.101),
    (1000, 1e-3), (1000, 0.05), (1000, 0.5), (1000, 0.97), (40000, 0.0003), (40000, 0.2),
    (10**6, 1e-6), (10**6, 2e-5), (10**6, 0.003), (10**6, 0.22), (10**6, 0.5),
]


def _chisq_pvalue(draws, n, p):
    draws = np.asarray(draws)
    lo, hi = int(draws.min()), int(draws.max())
    mu, sd = n * p, np.sqrt(n * p * (1 - p))
    lo = max(0, min(lo, int(mu - 8 * sd) - 1))
    hi = min(n, max(hi, int(mu + 8 * sd) + 1))
    ks = np.arange(lo, hi + 1)
    pmf = stats.binom.pmf(ks, n, p)
    # fold the outer tails into the end cells so the expected counts sum to len(draws)
    pmf[0] += stats.binom.cdf(lo - 1, n, p)
    pmf[-1] += stats.binom.sf(hi, n, p)
    obs = np.bincount(draws - lo, minlength=len(ks)).astype(np.float64)
    exp = pmf * len(draws)
    # merge cells with small expectation from both ends towards the middle
    o_m, e_m = [], []
    acc_o = acc_e = 0.0
    for o, e in zip(obs, exp):
        acc_o += o
        acc_e += e
        if acc_e >= 20:
            o_m.append(acc_o)
            e_m.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0:
        if e_m:
            o_m[-1] += acc_o
            e_m[-1] += acc_e
        else:
            o_m.append(acc_o)
            e_m.append(acc_e)
    o_m, e_m = np.array(o_m), np.array(e_m)
    if len(o_m) < 2:
        return 1.0
    chi2 = ((o_m - e_m) ** 2 / e_m).sum()
    return stats.chi2.sf(chi2, len(o_m) - 1)


@pytest.mark.parametrize("prec", [O.PREC_FP64, O.PREC_FP32])
@pytest.mark.parametrize("n,p", CELLS)
def test_binomial_matches_exact_pmf(prec, n, p):
    p_eff = float(np.float32(p)) if prec == O.PREC_FP32 else p
    x = O.binomial_batch(prec, n, p_eff, seed=1000 + n % 97, count=200_000, i=3, k=2, t=5, b=1)
    assert x.min() >= 0 and x.max() <= n
    pv = _chisq_pvalue(x, n, p_eff)
    assert pv > 1e-4, (n, p, prec, pv, x.mean(), n * p_eff)


@pytest.mark.parametrize("prec", [O.PREC_FP64, O.PREC_FP32])
def test_binomial_edge_cases(prec):
    for j in range(50):
        assert O.binomial(prec, 0, 0.3, 1, j, 0, 1, 1, 0) == 0
        assert O.binomial(prec, 17, 0.0, 1, j, 0, 1, 1, 0) == 0
        assert O.binomial(prec, 17, 1.0, 1, j, 0, 1, 1, 0) == 17
        assert O.binomial(prec, 10**6, 1.0, 1, j, 0, 1, 1, 0) == 10**6
        assert O.binomial(prec, -3, 0.5, 1, j, 0, 1, 1, 0) == 0


def test_binomial_streams_are_distinct():
    a = O.binomial_batch(O.PREC_FP64, 1000, 0.3, 5, 4000, i=0, k=1, t=1, b=0)
    b = O.binomial_batch(O.PREC_FP64, 1000, 0.3, 5, 4000, i=0, k=1, t=1, b=1)
    c = O.binomial_batch(O.PREC_FP64, 1000, 0.3, 5, 4000, i=1, k=1, t=1, b=0)
    d = O.binomial_batch(O.PREC_FP64, 1000, 0.3, 5, 4000, i=0, k=2, t=1, b=0)
    for other in (b, c, d):
        assert abs(np.corrcoef(a, other)[0, 1]) < 0.08
    # and deterministic
    assert np.array_equal(a, O.binomial_batch(O.PREC_FP64, 1000, 0.3, 5, 4000, i=0, k=1, t=1, b=0))


def test_poisson_logpmf():
    for lam in [1, 2, 7, 50, 1000, 123456]:
        for y in [0, 1, 3, 10, 49, 1000, 130000]:
            got = O.obs_logpmf(O.OBS_POIS_INC, y, lam)
            want = stats.poisson.logpmf(y, lam)
            assert got == pytest.approx(want, rel=1e-12, abs=1e-9), (y, lam)
    assert O.obs_logpmf(O.OBS_POIS_INC, 0, 0) == 0.0
    assert O.obs_logpmf(O.OBS_POIS_INC, 3, 0) == -np.inf


def test_negbin_logpmf():
    for r in [0.7, 3.0, 10.0, 55.5]:
        for mu in [1, 4, 60, 5000, 200000]:
            for y in [0, 1, 5, 63, 4000, 250000]:
                got = O.obs_logpmf(O.OBS_NB_INC, y, mu, r)
                want = stats.nbinom.logpmf(y, r, r / (r + mu))
                assert got == pytest.approx(want, rel=1e-11, abs=1e-8), (y, mu, r)
    assert O.obs_logpmf(O.OBS_NB_INC, 0, 0, 10.0) == 0.0
    assert O.obs_logpmf(O.OBS_NB_INC, 2, 0, 10.0) == -np.inf
