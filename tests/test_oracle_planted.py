"""Each pin catches the mistakes it is there for: copies of the CPU reference with one
plausible mistake planted (tests/planted.py) fail the pin that the reference passes.

* The age-structured force of infection lambda_g = beta s_g sum_h C_gh I_h / N_h
  (exact enumeration of a four-group population with a non-symmetric contact matrix,
  unequal groups and distinct susceptibilities): a transposed C, N_g in place of N_h,
  and s_h in place of s_g.
* The filter's weight recursion and likelihood increment (Sec. II, with the mean-weight
  reset after resampling) against the Kalman filter: a dropped log S_prev, S_prev not
  updated, no weight reset after resampling, log-weights not re-based on the maximum,
  and ancestors shifted by one slot.
* The population random walk's proposals and weights against their definitions: the
  proposal's density dropped from the weight, and the covariance taken without the
  population's weights.
* The p-MCMC acceptance (Sec. III, Eq. MHalgorithm_) against the exact grid posterior:
  the prior dropped from the ratio, and the current state's likelihood estimate drawn
  afresh every iteration instead of travelling with the state.
"""
import concurrent.futures as cf

import numpy as np
import pytest

from tests import planted as PL
from tests.test_oracle_kalman import kalman_pin_statistic
from tests.test_oracle_pf_exact import age_pin_statistic
from tests.test_oracle_pmcmc import pmcmc_pin_statistic

COEF = "mc.cs[g][h] = (REAL)(((beta * s[g]) * cfg->fixed[4 * g + h]) / ngs[h]);"
AGE_PLANTS = {
    "transposed_contact_matrix": [("pf_real.inc", COEF, COEF.replace("fixed[4 * g + h]", "fixed[4 * h + g]"))],
    "receiving_group_size": [("pf_real.inc", COEF, COEF.replace("/ ngs[h]", "/ ngs[g]"))],
    "source_susceptibility": [("pf_real.inc", COEF, COEF.replace("s[g])", "s[h])"))],
}
KALMAN_PLANTS = {
    "dropped_log_s_prev": [("pf_real.inc", "*inc = (((double)m + log(S)) - log(*s_prev)) + cst;",
                            "*inc = ((double)m + log(S)) + cst;")],
    "s_prev_not_updated": [("pf_real.inc", "    *s_prev = S;\n", "")],
    "no_weight_reset": [("pf_real.inc", "    for (int jj = 0; jj < nx; ++jj) lw[jj] = (REAL)0;\n", "")],
    "not_rebased_on_max": [("pf_real.inc", "lw[jj] = a[jj] - m;", "lw[jj] = a[jj];")],
    "ancestors_shifted": [("smc2_oracle.c", "        anc[m] = j;", "        anc[m] = j + 1 < n ? j + 1 : j;")],
}


SCORE_PLANTS = {
    # a particle keeps its own score when resampling hands it another trajectory's state
    "score_not_resampled": [("pf_real.inc", "                memcpy(sj, sjs, sizeof(double) * (size_t)nx * D);\n", ""),
                            ("smc2_oracle.c", "                memcpy(sj, sjs, sizeof(double) * (size_t)nx * 3);\n", "")],
    # the final average without the last day's weights
    "score_unweighted": [("pf_real.inc", "num = num + w[jj] * sj[(size_t)jj * D + d];",
                          "num = num + (S / (double)nx) * sj[(size_t)jj * D + d];"),
                         ("smc2_oracle.c", "num = num + w[j] * sj[(size_t)j * 3 + d];",
                          "num = num + (S / (double)nx) * sj[(size_t)j * 3 + d];")],
    # the infection flow's d h / d beta = I / N_pop dropped
    "hazard_derivative_dropped": [("pf_real.inc", "sc[0] = FN(flow_score)(S, p_si, nsi) * ((double)I / cfg->n_pop);",
                                   "sc[0] = FN(flow_score)(S, p_si, nsi);")],
}


LANGEVIN_PLANTS = {
    # the drifted proposal weighted as if it were the symmetric random walk
    "langevin_density_dropped": [("smc2_oracle.c", "(learned || drift) ? lq : NULL", "learned ? lq : NULL")],
    # log q evaluated around phi instead of the drifted mean phi + delta
    "langevin_density_undrifted": [("smc2_oracle.c", "    return or_mvn_logpdf_chol(D, phi_new, m, L);",
                                    "    return or_mvn_logpdf_chol(D, phi_new, phi, L);")],
}

RW_POP_PLANTS = {
    # the population random walk weighted with the fixed random walk's density
    "rw_pop_density_dropped": [("smc2_oracle.c", "(learned || drift) ? lq : NULL",
                                "(learned || (drift && lgv)) ? lq : NULL")],
    # the proposal covariance of the population with its weights ignored
    "rw_pop_unweighted_covariance": [("smc2_oracle.c", "for (int i = 0; i < N; ++i) wn[i] = exp(logw[i] - Wl);",
                                      "for (int i = 0; i < N; ++i) wn[i] = 1.0 / N;")],
}


PMCMC_PLANTS = {
    "prior_dropped_from_the_ratio": [("smc2_oracle.c", "    const double cur = lp + ll, nw = lp_new + ll_new;",
                                      "    const double cur = ll, nw = ll_new;")],
    # the current state's estimate refreshed every iteration (Monte Carlo within Metropolis)
    "estimate_not_kept": [("smc2_oracle.c", "                const int acc = or_mh_accept(lp, ll, lpn, lln, or_u53(w[0], w[1]));",
                           "                if (lp != -INFINITY) { or_theta_of_phi(cfg, phi, th); ll = or_pf_loglik(cfg, th, y, T, nx, "
                           "seed, (uint32_t)c, (uint32_t)(m + 40000), NULL, NULL); }\n"
                           "                const int acc = or_mh_accept(lp, ll, lpn, lln, or_u53(w[0], w[1]));")],
}


@pytest.fixture(scope="module")
def planted_libs(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("planted"))
    plants = dict(AGE_PLANTS, **KALMAN_PLANTS, **PMCMC_PLANTS, **SCORE_PLANTS, **LANGEVIN_PLANTS, **RW_POP_PLANTS)
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        futs = {name: ex.submit(PL.build_planted, name, edits, d) for name, edits in plants.items()}
        return {name: f.result() for name, f in futs.items()}


def test_the_reference_passes_both_pins():
    mean, se = age_pin_statistic()
    assert abs(mean - 1.0) < 4 * se, (mean, se)
    mean, se = kalman_pin_statistic()
    assert abs(mean - 1.0) < 4 * se + 1e-3, (mean, se)


@pytest.mark.parametrize("name", sorted(AGE_PLANTS))
def test_age_pin_catches_a_misread_force_of_infection(planted_libs, name):
    with PL.installed(planted_libs[name]):
        mean, se = age_pin_statistic()
    print(name, mean, se)
    assert abs(mean - 1.0) > 4 * se, (name, mean, se)


@pytest.mark.parametrize("name", sorted(KALMAN_PLANTS))
def test_kalman_pin_catches_a_broken_weight_recursion(planted_libs, name):
    with PL.installed(planted_libs[name]):
        mean, se = kalman_pin_statistic()
    print(name, mean, se)
    assert abs(mean - 1.0) > 4 * se + 1e-3, (name, mean, se)


@pytest.mark.parametrize("name", sorted(SCORE_PLANTS))
def test_score_pins_catch_a_broken_score(planted_libs, name):
    from tests.test_oracle_score import _close, lg_score_statistic, sir_score_statistic
    with PL.installed(planted_libs[name]):
        ok_sir = _close(*sir_score_statistic(M=100))[0]
        ok_lg = _close(*lg_score_statistic(M=100))[0]
    print(name, ok_sir, ok_lg)
    assert not (ok_sir and ok_lg), name


@pytest.mark.parametrize("name", sorted(LANGEVIN_PLANTS))
def test_langevin_pin_catches_an_inexact_weight(planted_libs, name):
    from tests.test_oracle_langevin import langevin_grid_statistic
    with PL.installed(planted_libs[name]):
        # at the full step the weight's error is large enough for the grid test to see; at
        # the default quarter step the proposal is nearly symmetric and the error small
        ests, second, grid_mean, grid_sd, _ = langevin_grid_statistic(step=1.0)
    se = ests.std(0, ddof=1) / np.sqrt(len(ests))
    pooled_sd = np.sqrt(second.mean(0) - ests.mean(0) ** 2)
    print(name, ests.mean(0), grid_mean, se, pooled_sd / grid_sd)
    assert np.any(np.abs(ests.mean(0) - grid_mean) > 4 * se + 2e-3) or np.any(np.abs(pooled_sd / grid_sd - 1) > 0.2)


@pytest.mark.parametrize("name", sorted(RW_POP_PLANTS))
def test_rw_pop_pin_catches_a_wrong_covariance_or_density(planted_libs, name):
    from tests.test_oracle_rwpop import rw_pop_discrepancies
    with PL.installed(planted_libs[name]):
        dphi, dlw, _, _ = rw_pop_discrepancies()
    print(name, dphi, dlw)
    assert dphi > 1e-6 or dlw > 1e-6, (name, dphi, dlw)


@pytest.mark.parametrize("name", sorted(PMCMC_PLANTS))
def test_pmcmc_pin_catches_a_wrong_acceptance(planted_libs, name):
    with PL.installed(planted_libs[name]):
        mean, se, sd, gm, gsd, rate = pmcmc_pin_statistic()
    print(name, mean, gm, se, sd, gsd)
    assert np.any(np.abs(mean - gm) > 4 * se + 2e-3) or np.any(np.abs(sd / gsd - 1) > 0.15), (name, mean, sd)
