"""Pins of the reference score estimator (Fisher's identity: the gradient of log p(y | theta)
is the posterior expectation of the complete-data score; each particle carries its
trajectory's score through resampling and the last day's weights average it).

The estimator is consistent in N_x, not unbiased (a ratio of weighted sums over
degenerating paths), so it is pinned at large N_x against exact gradients computed
independently: central differences of the Kalman log-likelihood for the linear-Gaussian
model, and of the enumerated exact likelihoods of tiny SIR and SEIR populations
(tests/exact_models.py), including the negative-binomial dispersion r. Copies with a
planted mistake fail these pins (tests/test_oracle_planted.py)."""
import numpy as np
import pytest
from scipy import special

import oracle as O
from paper_2311_12973_amd import workloads as W
from tests import exact_models as X
from tests.test_oracle_kalman import M0, PHI, S0, SQ, SR, kalman_loglik, simulate


def central_difference(f, x, h=1e-6):
    g = []
    for d in range(len(x)):
        xp = np.array(x, float)
        xm = np.array(x, float)
        xp[d] += h
        xm[d] -= h
        g.append((f(xp) - f(xm)) / (2 * h))
    return np.array(g)


def _close(sc, exact, rel_bias=0.005):
    """mean over filters within 4 s.e. plus a small allowance for the O(1/N_x) bias"""
    mean, se = sc.mean(0), sc.std(0, ddof=1) / np.sqrt(len(sc))
    tol = 4 * se + rel_bias * np.maximum(1.0, np.abs(exact))
    return np.all(np.abs(mean - exact) < tol), mean, se


def test_digamma_matches_scipy():
    for x in [1e-3, 0.3, 1.0, 2.5, 9.999, 10.0, 10.001, 37.2, 1e3, 1e6]:
        assert O.digamma(x) == pytest.approx(special.digamma(x), rel=1e-14, abs=1e-14), x


def lg_score_statistic(nx=4096, M=200):
    y = simulate(25, 11)
    exact = central_difference(lambda v: kalman_loglik(v[0], v[1], v[2], M0, S0, y), [PHI, SQ, SR], 1e-5)
    sc = np.array([O.pf_lg(PHI, SQ, SR, M0, S0, y, nx, 7, filt=f, score=True)[1] for f in range(M)])
    return sc, exact


def test_linear_gaussian_score_matches_the_kalman_gradient():
    sc, exact = lg_score_statistic()
    ok, mean, se = _close(sc, exact)
    assert ok, (mean, exact, se)


N_POP, I0, T, BETA, GAMMA = 16, 2, 6, 1.4, 0.35


def sir_score_statistic(obs=O.OBS_POIS_INC, prec=O.PREC_FP64, nx=8192, M=200):
    y = W.simulate(W.SIR, obs, N_POP, [BETA, GAMMA], T, seed=11, fixed=[I0], min_frac=0)
    exact = central_difference(lambda v: X.sir_loglik(v[0], v[1], N_POP, I0, y, obs), [BETA, GAMMA])
    cfg = O.make_config(O.SIR, obs, 2, prec, N_POP, [[O.PRIOR_UNIFORM, 0, 5]] * 2, np.eye(2), [I0])
    sc = np.array([O.pf_score(cfg, [BETA, GAMMA], y, nx, 1 + m, m % 7, 1)[1] for m in range(M)])
    return sc, exact


@pytest.mark.parametrize("obs,prec", [(O.OBS_POIS_INC, O.PREC_FP64), (O.OBS_POIS_PREV, O.PREC_FP64),
                                      (O.OBS_POIS_INC, O.PREC_FP32)])
def test_sir_score_converges_to_the_exact_gradient(obs, prec):
    sc, exact = sir_score_statistic(obs, prec)
    ok, mean, se = _close(sc, exact)
    assert ok, (mean, exact, se)


def test_small_filters_are_biased_and_the_bias_shrinks():
    # the path-space estimator is a ratio over degenerate paths: biased at small N_x
    sc64, exact = sir_score_statistic(nx=64, M=1000)
    sc8k, _ = sir_score_statistic(nx=8192, M=200)
    assert np.abs(sc64.mean(0) - exact).max() > 5 * np.abs(sc8k.mean(0) - exact).max()


def test_seir_score_with_the_dispersion_converges_to_the_exact_gradient():
    n_pop, T_, r = 8, 5, 3.0
    beta, sigma, gamma = 1.6, 0.5, 0.3
    iota = 2.0 / n_pop
    y = W.simulate(W.SEIR, W.OBS_NB_INC, n_pop, [beta, sigma, gamma, iota], T_, seed=21, fixed=[r], min_frac=0)
    exact = central_difference(lambda v: X.seir_loglik(v[0], v[1], v[2], n_pop, 2, y, v[3]), [beta, sigma, gamma, r])
    c5 = O.make_config(O.SEIR, O.OBS_NB_INC, 5, O.PREC_FP64, n_pop, [[O.PRIOR_UNIFORM, 0, 5]] * 5, np.eye(5), [])
    sc = np.array([O.pf_score(c5, [beta, sigma, gamma, iota, r], y, 2048, 1 + m, m % 7, 1)[1] for m in range(300)])
    assert np.all(sc[:, 3] == 0.0)  # iota: no score
    ok, mean, se = _close(sc[:, [0, 1, 2, 4]], exact)
    assert ok, (mean, exact, se)
    # with r fixed (D = 4) the first three coordinates are the same estimates
    c4 = O.make_config(O.SEIR, O.OBS_NB_INC, 4, O.PREC_FP64, n_pop, [[O.PRIOR_UNIFORM, 0, 5]] * 4, np.eye(4), [r])
    for m in range(3):
        _, s4 = O.pf_score(c4, [beta, sigma, gamma, iota], y, 2048, 1 + m, m % 7, 1)
        assert np.array_equal(s4[:3], sc[m, :3]) and s4[3] == 0.0


def test_score_filter_returns_the_filter_estimate():
    w = W.preset("seir")
    w["T"] = 30
    y = W.observations(w)
    cfg = O.config_from_workload(w)
    for i in range(3):
        ll, sc = O.pf_score(cfg, w["truth"], y, 128, 5, i, 2)
        assert ll == O.pf_loglik(cfg, w["truth"], y, 128, 5, i, 2)
        assert np.all(np.isfinite(sc)) and sc[3] == 0.0


def test_dead_filter_and_unsupported_model():
    w = W.preset("paper_sir")
    y = np.zeros((5, 1), dtype=np.int32)
    y[2, 0] = 3
    cfg = O.config_from_workload(dict(w, fixed=[0]))
    ll, sc = O.pf_score(cfg, [0.5, 0.2], y, 64, 1, 0, 1)
    assert ll == -np.inf and np.all(sc == 0.0)
    wa = W.preset("age_seir")
    ll, sc = O.pf_score(O.config_from_workload(wa), wa["truth"], W.observations(dict(wa, T=5)), 16, 1, 0, 1)
    assert np.isnan(ll) and np.all(np.isnan(sc))
