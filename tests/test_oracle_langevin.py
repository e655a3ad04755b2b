"""Pins of the reference truncated Langevin proposal (a gradient-informed proposal for
Sec. IV-A's q, using the particle filter's score estimate; the estimate travels with its
sample, so q stays an exact density and Eq. l_weights exact).

* With a flat prior and a zero score the drift vanishes: the proposal is the random
  walk's (same normals) and log q its Gaussian density (scipy).
* The drift equals the step fraction (1/4 by default) times 1/2 Sigma times the gradient
  on the sampler coordinates of s . theta(phi) + log prior(phi), taken by central
  differences of the reference's own coordinate map and prior density (the chain rule
  and the prior's gradient are not retyped).
* A large score's drift is shrunk to Mahalanobis length 1 before the step fraction: its
  length is the fraction.
* The sampler with it reaches the exact grid posterior of the tiny SIR problem; copies
  that weight it as the symmetric random walk, or leave the scores behind when the
  population is resampled, do not (tests/test_oracle_planted.py).
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from paper_2311_12973_amd import workloads as W
from tests.test_oracle_mlp import I0, MED, N_POP, SD, _grid_posterior


def _rw_cov(cfg):
    return np.array([[cfg.rw_cov[a][c] for c in range(cfg.D)] for a in range(cfg.D)])


def test_zero_score_with_a_flat_prior_is_the_random_walk():
    w = W.preset("paper_sir")
    cfg = O.config_from_workload(w)
    phi = np.array([[0.6, 0.3], [0.2, 0.7], [0.9, 0.1]])
    rw = O.propose_rw(cfg, 5, 3, phi)[0]
    for i in range(3):
        pn, lq = O.propose_langevin(cfg, phi[i], np.zeros(2), 5, 3, i)
        assert np.array_equal(pn, rw[i])
        assert lq == pytest.approx(stats.multivariate_normal(phi[i], _rw_cov(cfg)).logpdf(pn), rel=1e-12)


def _fd_grad(f, x, h=1e-6):
    g = np.zeros(len(x))
    for d in range(len(x)):
        e = np.zeros(len(x))
        e[d] = h
        g[d] = (f(x + e) - f(x - e)) / (2 * h)
    return g


@pytest.mark.parametrize("name,step", [("seir", 0.0), ("seir_learned", 0.0), ("lingauss", 0.0), ("seir", 1.0),
                                       ("lingauss", 0.5)])
def test_drift_is_half_sigma_times_the_gradient(name, step):
    w = dict(W.preset(name), lgv_step=step)
    cfg = O.config_from_workload(w)
    rng = np.random.default_rng(3)
    for i in range(4):
        th = np.array(w["truth"]) * np.exp(rng.normal(0, 0.05, w["D"]))
        phi = np.array([np.log(t) if p[0] == O.PRIOR_LOGNORMAL else
                        (np.log(t / (1 - t)) if p[0] == O.PRIOR_LOGITNORMAL else t) for t, p in zip(th, w["prior"])])
        s = rng.normal(0, 0.5, w["D"]) / np.maximum(np.abs(th), 1e-3) * 1e-2  # small: no truncation
        pn, _ = O.propose_langevin(cfg, phi, s, 7, 2, i)
        lz = O.propose_rw(cfg, 7, 2, np.tile(phi, (i + 1, 1)))[0][i] - phi
        grad = _fd_grad(lambda p: float(s @ O.theta_of_phi(cfg, p)) + O.prior_logpdf(cfg, p), phi)
        full = 0.5 * _rw_cov(cfg) @ grad
        assert np.linalg.norm(np.linalg.solve(np.linalg.cholesky(_rw_cov(cfg)), full)) < 1.0
        drift = (step if step > 0 else 0.25) * full
        assert np.allclose(pn - phi - lz, drift, rtol=1e-6, atol=1e-9), (pn - phi - lz, drift)


@pytest.mark.parametrize("step", [0.0, 1.0])
def test_large_drift_is_truncated_to_unit_mahalanobis_length(step):
    w = dict(W.preset("seir"), lgv_step=step)
    cfg = O.config_from_workload(w)
    phi = np.array([np.log(0.5), np.log(0.25), np.log(0.2), np.log(2e-5 / (1 - 2e-5))])
    L = np.linalg.cholesky(_rw_cov(cfg))
    lz = O.propose_rw(cfg, 7, 2, phi[None, :])[0][0] - phi
    for s in ([1e4, 0, 0, 0], [-300.0, 50.0, 2e3, 1e5]):
        pn, lq = O.propose_langevin(cfg, phi, np.array(s), 7, 2, 0)
        drift = pn - phi - lz
        assert np.linalg.norm(np.linalg.solve(L, drift)) == pytest.approx(step if step > 0 else 0.25, rel=1e-12)
        assert lq == pytest.approx(stats.multivariate_normal(phi + drift, _rw_cov(cfg)).logpdf(pn), rel=1e-10)


def langevin_grid_statistic(seeds=12, N=1024, K=8, step=0.0):
    y, grid_mean, grid_sd = _grid_posterior()
    prior = [[O.PRIOR_LOGNORMAL, np.log(MED[0]), SD], [O.PRIOR_LOGNORMAL, np.log(MED[1]), SD]]
    cfg = O.make_config(O.SIR, O.OBS_POIS_PREV, 2, O.PREC_FP64, N_POP, prior, 0.05 * np.eye(2), [I0],
                        lkernel=O.L_FORWARD, proposal=O.PROP_LANGEVIN, lgv_step=step)
    ests, second, used = [], [], 0
    for seed in range(1, seeds + 1):
        out = O.smc2_run(cfg, y, nx=48, seed=seed, N=N, K=K)
        assert out["status"] == 0
        used += int((out["rec"][1:, -2] == 2).sum())
        mean, cov, _ = O.recycle(out["rec"], 2)
        ests.append(mean)
        second.append(np.diag(cov) + mean ** 2)
    ests = np.array(ests)
    return ests, np.array(second), grid_mean, grid_sd, used


@pytest.mark.parametrize("step", [0.0, 1.0])
def test_langevin_sampler_targets_the_grid_posterior(step):
    """With the forward-kernel setting each Langevin iteration is weighted through the
    random walk's backward kernel and the proposal's exact density (Eq. l_weights)."""
    ests, second, grid_mean, grid_sd, used = langevin_grid_statistic(step=step)
    assert used == 12 * 7
    se = ests.std(0, ddof=1) / np.sqrt(len(ests))
    assert np.all(np.abs(ests.mean(0) - grid_mean) < 4 * se + 2e-3), (ests.mean(0), grid_mean, se)
    pooled_sd = np.sqrt(second.mean(0) - ests.mean(0) ** 2)
    assert np.all(np.abs(pooled_sd / grid_sd - 1) < 0.2), (pooled_sd, grid_sd)
