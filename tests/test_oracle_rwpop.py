"""Pins of the reference random walk with the population's covariance (PROP_RW_POP): a
Gaussian q for Sec. IV-A whose covariance is the weighted covariance of the proposing
population, with its density in Eq. l_weights.

* Each proposal of iteration k >= 2 is phi + L z: z the random walk's normals of the same
  sample and iteration, L L' the weighted covariance of the population after iteration
  k - 1, formed here with numpy from the dumped proposals, ancestors and weights (not the
  reference's frame routine); a collapsed population (one distinct sample after a
  resampling) falls back to the diagonal of the standard deviations, floored at 1e-6.
* The pre-resampling log-weights are Eq. l_weights with the forward-kernel setting's
  backward kernel N(phi_{k-1}; phi_k, Sigma_RW) and q = N(phi_k; phi_{k-1}, Sigma_pop),
  both taken from scipy.
* The sampler reaches the exact grid posterior of the tiny SIR problem with either
  L-kernel; a copy that weights it with the fixed random walk's density does not
  (tests/test_oracle_planted.py).
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from paper_2311_12973_amd import workloads as W
from tests.test_oracle_mlp import I0, MED, N_POP, SD, _grid_posterior


def _rw_cov(cfg):
    return np.array([[cfg.rw_cov[a][c] for c in range(cfg.D)] for a in range(cfg.D)])


def _factor(C, mu):
    """Cholesky factor of the population covariance C; for a degenerate population (a
    pivot not above 1e-12 of its coordinate's raw second moment, e.g. every sample a copy
    of one after a collapse) the diagonal of the standard deviations, floored at 1e-6."""
    try:
        L = np.linalg.cholesky(C)
        if np.all(np.diag(L) ** 2 > 1e-12 * (np.diag(C) + mu ** 2)):
            return L
    except np.linalg.LinAlgError:
        pass
    return np.diag(np.maximum(np.sqrt(np.diag(C)), 1e-6))


def rw_pop_discrepancies(name="seir", N=96, K=4, nx=40, T=5, seed=5):
    """Largest differences of the reference sampler's proposals and pre-resampling
    log-weights (iterations 2..K) from their definitions, the number of iterations
    checked and how many of them proposed from a population that was not resampled
    (unequal weights). At T = 5 the first SEIR iteration keeps its weights (ESS 58 of
    96)."""
    w = dict(W.preset(name), proposal=O.PROP_RW_POP, lkernel=O.L_FORWARD, T=T)
    y = W.observations(w)
    cfg = O.config_from_workload(w)
    ref = O.smc2_run(cfg, y, nx, seed, N, K, dumps=True)
    assert ref["status"] == 0
    D = w["D"]
    Lrw = np.linalg.cholesky(_rw_cov(cfg))
    dphi, dlw, checked, weighted = 0.0, 0.0, 0, 0
    for k in range(2, K + 1):
        anc = ref["anc"][k - 2]
        phi = ref["phi"][k - 2][anc]
        lp, ll = ref["lp"][k - 2][anc], ref["ll"][k - 2][anc]
        logw = np.zeros(N) if ref["rec"][k - 2, 2] else ref["logw"][k - 2][anc]
        weighted += int(np.ptp(logw[np.isfinite(logw)]) > 0)
        wn = np.exp(logw - logw.max())
        wn /= wn.sum()
        mu = wn @ phi
        C = (phi - mu).T @ ((phi - mu) * wn[:, None])
        L = _factor(C, mu)
        S = L @ L.T
        z = np.linalg.solve(Lrw, (O.propose_rw(cfg, seed, k, phi)[0] - phi).T).T
        phin = ref["phi"][k - 1]
        dphi = max(dphi, float(np.abs(phin - (phi + z @ L.T)).max()))
        for i in range(N):
            pin = ref["lp"][k - 1][i] + ref["ll"][k - 1][i]
            if not np.isfinite(pin) or not np.isfinite(logw[i]):
                assert ref["logw"][k - 1][i] == -np.inf
                continue
            lL = stats.multivariate_normal(phin[i], _rw_cov(cfg)).logpdf(phi[i])
            lq = stats.multivariate_normal(phi[i], S).logpdf(phin[i])
            want = logw[i] + pin - (lp[i] + ll[i]) + lL - lq
            dlw = max(dlw, abs(ref["logw"][k - 1][i] - want) / max(1.0, abs(want)))
        assert np.all(ref["rec"][k - 1, -2] == 3)
        checked += 1
    assert ref["rec"][0, -2] == 0
    return dphi, dlw, checked, weighted


@pytest.mark.parametrize("name,T", [("seir", 5), ("sir_fp64", 25), ("seir_learned", 25)])
def test_proposals_and_weights_follow_the_population_covariance(name, T):
    dphi, dlw, checked, weighted = rw_pop_discrepancies(name, T=T)
    assert checked == 3
    if name == "seir":
        assert weighted >= 1
    assert dphi < 1e-9, dphi
    assert dlw < 1e-9, dlw


def rw_pop_grid_statistic(lkernel, seeds=12, N=1024, K=8):
    y, grid_mean, grid_sd = _grid_posterior()
    prior = [[O.PRIOR_LOGNORMAL, np.log(MED[0]), SD], [O.PRIOR_LOGNORMAL, np.log(MED[1]), SD]]
    cfg = O.make_config(O.SIR, O.OBS_POIS_PREV, 2, O.PREC_FP64, N_POP, prior, 0.05 * np.eye(2), [I0],
                        lkernel=lkernel, proposal=O.PROP_RW_POP)
    ests, second = [], []
    for seed in range(1, seeds + 1):
        out = O.smc2_run(cfg, y, nx=48, seed=seed, N=N, K=K)
        assert out["status"] == 0
        assert np.all(out["rec"][1:, -2] == 3)
        mean, cov, _ = O.recycle(out["rec"], 2)
        ests.append(mean)
        second.append(np.diag(cov) + mean ** 2)
    return np.array(ests), np.array(second), grid_mean, grid_sd


@pytest.mark.parametrize("lkernel", [O.L_FORWARD, O.L_GAUSS_OPT])
def test_population_walk_targets_the_grid_posterior(lkernel):
    ests, second, grid_mean, grid_sd = rw_pop_grid_statistic(lkernel)
    se = ests.std(0, ddof=1) / np.sqrt(len(ests))
    print(lkernel, ests.mean(0), grid_mean, se)
    assert np.all(np.abs(ests.mean(0) - grid_mean) < 4 * se + 2e-3), (ests.mean(0), grid_mean, se)
    pooled_sd = np.sqrt(second.mean(0) - ests.mean(0) ** 2)
    assert np.all(np.abs(pooled_sd / grid_sd - 1) < 0.2), (pooled_sd, grid_sd)
