"""End-to-end pin of the reference SMC^2 sampler against an exact grid posterior.

A tiny SIR epidemic (Sec. V-A model with Poisson observations of prevalence) has an
exact likelihood (tests/exact_models.py); on a grid it gives the exact posterior mean
of (beta, gamma). SMC^2 with particle-filter likelihoods targets that posterior
exactly (pseudo-marginal), so the mean over independent runs of its recycled
estimate (Sec. IV-C) must agree with the grid mean within Monte-Carlo error.

The sampler moves on unconstrained coordinates (log beta, log gamma with Gaussian
priors). With the paper's bounded U[0,1]^2 prior a Gaussian L-kernel puts mass
outside the support and the iterations k > 1 are biased towards the interior; only
the k = 1 importance-sampling step is exact there (test_uniform_prior_first_iteration).
"""
import numpy as np
import pytest

import oracle as O
from paper_2311_12973_amd import workloads as W
from tests import exact_models as X

N_POP, I0, T = 12, 2, 5
TRUTH = [0.85, 0.2]
MED, SD = (0.8, 0.2), 0.5


@pytest.fixture(scope="module")
def data():
    return W.simulate(W.SIR, W.OBS_POIS_PREV, N_POP, TRUTH, T, seed=4, fixed=[I0], min_frac=0)


@pytest.fixture(scope="module")
def problem(data):
    G = 80
    pb = np.log(MED[0]) + SD * np.linspace(-5.5, 5.5, G)
    pg = np.log(MED[1]) + SD * np.linspace(-5.5, 5.5, G)
    ll = X.sir_grid_loglik(np.exp(pb), np.exp(pg), N_POP, I0, data, X.POIS_PREV)
    lpri = -0.5 * ((pb[:, None] - np.log(MED[0])) / SD) ** 2 - 0.5 * ((pg[None, :] - np.log(MED[1])) / SD) ** 2
    lw = ll + lpri
    w = np.exp(lw - lw.max())
    w /= w.sum()
    mean = np.array([(w * np.exp(pb)[:, None]).sum(), (w * np.exp(pg)[None, :]).sum()])
    return data, mean


@pytest.mark.parametrize("lkernel", [O.L_GAUSS_OPT, O.L_FORWARD])
def test_recycled_posterior_mean_matches_grid(problem, lkernel):
    y, grid_mean = problem
    prior = [[O.PRIOR_LOGNORMAL, np.log(MED[0]), SD], [O.PRIOR_LOGNORMAL, np.log(MED[1]), SD]]
    cfg = O.make_config(O.SIR, O.OBS_POIS_PREV, 2, O.PREC_FP64, N_POP, prior, 0.05 * np.eye(2), [I0],
                        lkernel=lkernel)
    ests = []
    for seed in range(1, 13):
        out = O.smc2_run(cfg, y, nx=48, seed=seed, N=2048, K=8)
        assert out["status"] == 0
        mean, cov, c = O.recycle(out["rec"], 2)
        assert abs(c.sum() - 1) < 1e-12
        ests.append(mean)
    ests = np.array(ests)
    se = ests.std(0, ddof=1) / np.sqrt(len(ests))
    err = np.abs(ests.mean(0) - grid_mean)
    assert np.all(err < 4 * se + 2e-3), (ests.mean(0), grid_mean, se)


def test_uniform_prior_first_iteration(data):
    """The paper's U[0,1]^2 prior: the k = 1 importance-sampling estimate (q_1 = prior,
    w_1 = likelihood estimate, Eq. init_weights) is consistent for the posterior mean."""
    G = 80
    grid = (np.arange(G) + 0.5) / G
    ll = X.sir_grid_loglik(grid, grid, N_POP, I0, data, X.POIS_PREV)
    w = np.exp(ll - ll.max())
    w /= w.sum()
    gm = np.array([(w.sum(1) * grid).sum(), (w.sum(0) * grid).sum()])
    cfg = O.make_config(O.SIR, O.OBS_POIS_PREV, 2, O.PREC_FP64, N_POP, [[O.PRIOR_UNIFORM, 0.0, 1.0]] * 2,
                        0.02 * np.eye(2), [I0])
    m1 = np.array([O.smc2_run(cfg, data, nx=48, seed=s, N=4096, K=1)["rec"][0, 6:8] for s in range(1, 9)])
    se = m1.std(0, ddof=1) / np.sqrt(len(m1))
    assert np.all(np.abs(m1.mean(0) - gm) < 4 * se + 2e-3), (m1.mean(0), gm, se)


def test_run_dumps_are_consistent(data):
    y = data
    cfg = O.make_config(O.SIR, O.OBS_POIS_PREV, 2, O.PREC_FP64, N_POP, [[O.PRIOR_UNIFORM, 0.0, 1.0]] * 2,
                        0.02 * np.eye(2), [I0])
    out = O.smc2_run(cfg, y, nx=32, seed=3, N=64, K=4, dumps=True)
    again = O.smc2_run(cfg, y, nx=32, seed=3, N=64, K=4, dumps=True, n_threads=1)
    for key in ("phi", "ll", "lp", "logw", "anc", "rec"):
        assert np.array_equal(out[key], again[key])  # deterministic, thread-count invariant
    # iteration 1: log w = log-likelihood estimate (q_1 = prior)
    assert np.array_equal(out["logw"][0], out["ll"][0])
    # each particle filter log-likelihood matches a direct call at the same coordinates
    for i in range(0, 64, 9):
        th = O.theta_of_phi(cfg, out["phi"][2, i])
        assert O.pf_loglik(cfg, th, y, 32, 3, i, 3) == out["ll"][2, i] or not np.isfinite(out["ll"][2, i])
