"""Pins of the reference particle marginal Metropolis-Hastings (Sec. III, Eq.
MHalgorithm_), the paper's comparison method.

* The acceptance rule's special cases: a proposal with zero target is never accepted,
  one from a state with zero target always is, equal targets always are (u < 1).
* The chain targets the exact posterior whatever the number of particles (the estimate
  travels with its state): on the tiny SIR problem of the SMC^2 grid test, with noisy
  four-particle estimates (where a chain that drew its estimate afresh would be biased), the
  post-burn-in means of independent chains average to the exact grid posterior mean
  within four standard errors (from the spread across chains), and their pooled spread
  matches the grid's. Copies with a planted mistake (tests/test_oracle_planted.py) fail it.
* Chains are independent streams: a chain's trace does not depend on how many chains run.
"""
import numpy as np
import pytest

import oracle as O
from tests.test_oracle_mlp import MED, SD, _grid_posterior

N_POP, I0 = 12, 2


def test_acceptance_rule_special_cases():
    assert not O.mh_accept(-3.0, -10.0, -3.0, -np.inf, 0.5)
    assert not O.mh_accept(-3.0, -10.0, -np.inf, -5.0, 0.5)
    assert O.mh_accept(-3.0, -np.inf, -3.0, -50.0, 0.999999)
    assert O.mh_accept(-3.0, -10.0, -3.0, -10.0, 1 - 2.0**-53)
    # log u < difference of the log targets
    assert O.mh_accept(-1.0, -10.0, -1.0, -10.5, 0.6) == (np.log(0.6) < -0.5)
    assert O.mh_accept(-1.0, -10.0, -1.0, -10.5, 0.61) == (np.log(0.61) < -0.5)


def pmcmc_pin_statistic(chains=64, iters=600, burn=150, nx=4, seed=3):
    """(mean over chains of the post-burn-in means, their standard error, pooled posterior
    sd, grid mean, grid sd) for the tiny SIR problem with log-normal priors."""
    y, grid_mean, grid_sd = _grid_posterior()
    prior = [[O.PRIOR_LOGNORMAL, np.log(MED[0]), SD], [O.PRIOR_LOGNORMAL, np.log(MED[1]), SD]]
    cfg = O.make_config(O.SIR, O.OBS_POIS_PREV, 2, O.PREC_FP64, N_POP, prior, 0.1 * np.eye(2), [I0])
    th, ll, acc = O.pmcmc_run(cfg, y, nx, seed, chains, iters)
    post = th[:, 1 + burn:, :]
    cm = post.mean(1)
    se = cm.std(0, ddof=1) / np.sqrt(chains)
    pooled_sd = post.reshape(-1, 2).std(0)
    return cm.mean(0), se, pooled_sd, grid_mean, grid_sd, acc.mean()


@pytest.mark.slow
def test_pmcmc_targets_the_grid_posterior():
    mean, se, sd, gm, gsd, rate = pmcmc_pin_statistic()
    assert 0.05 < rate < 0.95
    assert np.all(np.abs(mean - gm) < 4 * se + 2e-3), (mean, gm, se)
    assert np.all(np.abs(sd / gsd - 1) < 0.15), (sd, gsd)


def test_chains_are_independent_of_their_number():
    y, _, _ = _grid_posterior()
    prior = [[O.PRIOR_LOGNORMAL, np.log(MED[0]), SD], [O.PRIOR_LOGNORMAL, np.log(MED[1]), SD]]
    cfg = O.make_config(O.SIR, O.OBS_POIS_PREV, 2, O.PREC_FP64, N_POP, prior, 0.1 * np.eye(2), [I0])
    a = O.pmcmc_run(cfg, y, 16, 9, 3, 20)
    b = O.pmcmc_run(cfg, y, 16, 9, 7, 20)
    for x, z in zip(a, b):
        assert np.array_equal(x, z[:3])
    th, ll, acc = a
    # a rejected proposal leaves the state and its estimate unchanged
    for c in range(3):
        for m in range(20):
            if not acc[c, m]:
                assert np.array_equal(th[c, m + 1], th[c, m]) and ll[c, m + 1] == ll[c, m]
            else:
                assert not np.array_equal(th[c, m + 1], th[c, m])
