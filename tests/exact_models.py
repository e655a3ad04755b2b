"""Exact marginal likelihoods of tiny chain-binomial epidemics (forward algorithm).

An independent third implementation used only to pin the reference particle
filter: it enumerates every compartment state and every flow, with the exact
binomial, Poisson and negative-binomial pmfs from scipy, so that
Z(theta) = p(y_{1:T} | theta) is exact up to FP64 rounding. The model is the
chain-binomial SIR of Sec. V-A (flows drawn from the previous day's state,
p(S->I) = 1 - exp(-beta I / N_pop), p(I->R) = 1 - exp(-gamma)) and its SEIR
extension; the observation is Poisson on prevalence (Sec. V-A) or on new cases, or
negative binomial on new cases.
"""
import math

import numpy as np
from scipy import stats

POIS_PREV, POIS_INC, NB_INC = 0, 1, 2


def _obs_pmf(obs, y, count, r):
    count = np.asarray(count, dtype=np.float64)
    if obs == NB_INC:
        out = np.where(count > 0, stats.nbinom.pmf(y, r, r / (r + np.maximum(count, 1e-300))), 0.0)
    else:
        out = np.where(count > 0, stats.poisson.pmf(y, np.maximum(count, 1e-300)), 0.0)
    return np.where(count > 0, out, 1.0 if y == 0 else 0.0)


def sir_loglik(beta, gamma, n_pop, i0, y, obs=POIS_INC):
    """log p(y | beta, gamma) for the SIR model with integer population n_pop."""
    n = int(n_pop)
    alpha = np.zeros((n + 1, n + 1))
    alpha[n - i0, i0] = 1.0
    p_ir = -math.expm1(-gamma)
    logZ = 0.0
    for yt in np.asarray(y).reshape(-1):
        new = np.zeros_like(alpha)
        for S in range(n + 1):
            for I in range(n + 1 - S):
                a = alpha[S, I]
                if a == 0.0:
                    continue
                p_si = -math.expm1(-beta * I / n_pop)
                f1 = stats.binom.pmf(np.arange(S + 1), S, p_si)
                f2 = stats.binom.pmf(np.arange(I + 1), I, p_ir)
                for nsi in range(S + 1):
                    if f1[nsi] == 0.0:
                        continue
                    for nir in range(I + 1):
                        pr = a * f1[nsi] * f2[nir]
                        if pr == 0.0:
                            continue
                        S2, I2 = S - nsi, I + nsi - nir
                        cnt = I2 if obs == POIS_PREV else nsi
                        new[S2, I2] += pr * float(_obs_pmf(obs, int(yt), cnt, 0.0))
        z = new.sum()
        if z == 0.0:
            return -np.inf
        logZ += math.log(z)
        alpha = new / z
    return logZ


def seir_loglik(beta, sigma, gamma, n_pop, i0, y, r, obs=NB_INC):
    """log p(y | theta) for the SEIR model (new cases = E->I flow)."""
    n = int(n_pop)
    alpha = {(n - i0, 0, i0): 1.0}
    p_ei = -math.expm1(-sigma)
    p_ir = -math.expm1(-gamma)
    logZ = 0.0
    for yt in np.asarray(y).reshape(-1):
        new = {}
        for (S, E, I), a in alpha.items():
            p_se = -math.expm1(-beta * I / n_pop)
            f1 = stats.binom.pmf(np.arange(S + 1), S, p_se)
            f2 = stats.binom.pmf(np.arange(E + 1), E, p_ei)
            f3 = stats.binom.pmf(np.arange(I + 1), I, p_ir)
            g = _obs_pmf(obs, int(yt), np.arange(E + 1), r)
            for nse in range(S + 1):
                for nei in range(E + 1):
                    w12 = a * f1[nse] * f2[nei] * g[nei]
                    if w12 == 0.0:
                        continue
                    for nir in range(I + 1):
                        pr = w12 * f3[nir]
                        if pr == 0.0:
                            continue
                        key = (S - nse, E + nse - nei, I + nei - nir)
                        new[key] = new.get(key, 0.0) + pr
        z = sum(new.values())
        if z == 0.0:
            return -np.inf
        logZ += math.log(z)
        alpha = {k: v / z for k, v in new.items()}
    return logZ


def sir_grid_loglik(betas, gammas, n_pop, i0, y, obs=POIS_PREV):
    """Exact log-likelihood on a grid of (beta, gamma), vectorised over the grid."""
    n = int(n_pop)
    B, G = np.meshgrid(np.asarray(betas, float), np.asarray(gammas, float), indexing="ij")
    B, G = B.ravel(), G.ravel()
    M = B.size
    alpha = np.zeros((M, n + 1, n + 1))
    alpha[:, n - i0, i0] = 1.0
    p_ir = -np.expm1(-G)
    logZ = np.zeros(M)
    for yt in np.asarray(y).reshape(-1):
        new = np.zeros_like(alpha)
        for S in range(n + 1):
            for I in range(n + 1 - S):
                a = alpha[:, S, I]
                if not np.any(a):
                    continue
                p_si = -np.expm1(-B * I / n_pop)
                f1 = stats.binom.pmf(np.arange(S + 1)[None, :], S, p_si[:, None])
                f2 = stats.binom.pmf(np.arange(I + 1)[None, :], I, p_ir[:, None])
                for nsi in range(S + 1):
                    for nir in range(I + 1):
                        S2, I2 = S - nsi, I + nsi - nir
                        cnt = I2 if obs == POIS_PREV else nsi
                        g = float(_obs_pmf(obs, int(yt), cnt, 0.0))
                        if g == 0.0:
                            continue
                        new[:, S2, I2] += a * f1[:, nsi] * f2[:, nir] * g
        z = new.sum(axis=(1, 2))
        with np.errstate(divide="ignore", invalid="ignore"):
            logZ += np.log(z)
            alpha = np.where(z[:, None, None] > 0, new / np.where(z > 0, z, 1.0)[:, None, None], 0.0)
    return logZ.reshape(len(betas), len(gammas))
