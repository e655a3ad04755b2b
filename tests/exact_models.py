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


def _group_states(n):
    """Every (S, E, I) with S + E + I <= n (R implied), and their index."""
    st = [(S, E, I) for S in range(n + 1) for E in range(n + 1 - S) for I in range(n + 1 - S - E)]
    return st, {s: a for a, s in enumerate(st)}


def age_seir_loglik_coef(A, group_sizes, i0, sigma, gamma, y, r):
    """log p(y | theta) for the four-group chain-binomial SEIR whose per-susceptible
    daily infection probability in group g is 1 - exp(-lambda_g) with
    lambda_g = sum_h A[g, h] I_h (previous day's infected), E->I and I->R as in the
    one-group SEIR, and y[t, g] ~ NB(mean = new cases E->I of group g, dispersion r).
    Groups are independent given the previous day's joint state, so one day's
    transition of the joint distribution is sum_x alpha(x) prod_g K_g(x, x'_g), with
    K_g the group's flow probabilities times its observation pmf."""
    A = np.asarray(A, dtype=np.float64)
    G = len(group_sizes)
    sts, idx = zip(*[_group_states(int(n)) for n in group_sizes])
    dims = [len(s) for s in sts]
    X = int(np.prod(dims))
    # own-state index of every joint state, per group, and that state's counts
    own = np.indices(dims).reshape(G, X)
    Icnt = [np.array([s[2] for s in sts[g]])[own[g]] for g in range(G)]
    p_ei = -math.expm1(-sigma)
    p_ir = -math.expm1(-gamma)
    alpha = np.zeros(X)
    start = [idx[g][(int(group_sizes[g]) - int(i0[g]), 0, int(i0[g]))] for g in range(G)]
    alpha[np.ravel_multi_index(start, dims)] = 1.0
    logZ = 0.0
    for yt in np.asarray(y).reshape(-1, G):
        lam = [sum(A[g, h] * Icnt[h] for h in range(G)) for g in range(G)]
        K = []
        for g in range(G):
            Kg = np.zeros((X, dims[g]))
            p_se = -np.expm1(-lam[g])
            for a, (S, E, I) in enumerate(sts[g]):
                rows = np.flatnonzero(own[g] == a)
                f1 = stats.binom.pmf(np.arange(S + 1)[None, :], S, p_se[rows][:, None])
                f2 = stats.binom.pmf(np.arange(E + 1), E, p_ei)
                f3 = stats.binom.pmf(np.arange(I + 1), I, p_ir)
                obs = _obs_pmf(NB_INC, int(yt[g]), np.arange(E + 1), r)
                for nse in range(S + 1):
                    for nei in range(E + 1):
                        for nir in range(I + 1):
                            c = f2[nei] * f3[nir] * obs[nei]
                            if c == 0.0:
                                continue
                            b = idx[g][(S - nse, E + nse - nei, I + nei - nir)]
                            Kg[rows, b] += f1[:, nse] * c
            K.append(Kg)
        new = np.zeros((dims[0] * dims[1], dims[2] * dims[3]))
        live = np.flatnonzero(alpha)
        for c0 in range(0, live.size, 4096):
            x = live[c0:c0 + 4096]
            m12 = (alpha[x, None, None] * K[0][x, :, None] * K[1][x, None, :]).reshape(x.size, -1)
            m34 = (K[2][x, :, None] * K[3][x, None, :]).reshape(x.size, -1)
            new += m12.T @ m34
        z = new.sum()
        if z == 0.0:
            return -np.inf
        logZ += math.log(z)
        alpha = new.reshape(-1) / z
    return logZ


def age_seir_loglik(beta, s, C, group_sizes, i0, sigma, gamma, y, r):
    """The age-structured SEIR's exact log-likelihood with the force of infection
    lambda_g = beta s_g sum_h C[g, h] I_h / N_h (susceptibility of the receiving group,
    contacts of g with h, prevalence in h)."""
    s = np.asarray(s, dtype=np.float64)
    N = np.asarray(group_sizes, dtype=np.float64)
    A = beta * s[:, None] * np.asarray(C, dtype=np.float64) / N[None, :]
    return age_seir_loglik_coef(A, group_sizes, i0, sigma, gamma, y, r)


def kalman_loglik_grid(a, sx, sy, m0, s0, y):
    """Exact log p(y_{1:T}) of the scalar linear-Gaussian model x_0 ~ N(m0, s0^2),
    x_t = a x_{t-1} + sx e_t, y_t = x_t + sy d_t (Kalman filter, prediction-error
    decomposition), vectorised over broadcastable parameter arrays a, sx, sy."""
    a, sx, sy = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (a, sx, sy)))
    m = np.full(a.shape, float(m0))
    P = np.full(a.shape, float(s0) ** 2)
    ll = np.zeros(a.shape)
    for yt in np.asarray(y, dtype=np.float64):
        m = a * m
        P = a * a * P + sx * sx
        S = P + sy * sy
        v = yt - m
        ll += -0.5 * (np.log(2.0 * np.pi * S) + v * v / S)
        K = P / S
        m = m + K * v
        P = (1.0 - K) * P
    return ll


def lingauss_loglik_joint(a, sx, sy, m0, s0, y):
    """The same likelihood from the joint Gaussian of y_{1:T}: mean a^t m0 and covariance
    a^(s+t) s0^2 + sx^2 sum_{u <= min(s,t)} a^(s-u) a^(t-u) + sy^2 [s = t]."""
    from scipy import stats as st
    y = np.asarray(y, dtype=np.float64)
    T = y.shape[0]
    t = np.arange(1, T + 1)
    mean = a ** t * m0
    cov = np.empty((T, T))
    for i in range(T):
        for j in range(T):
            s_, t_ = i + 1, j + 1
            acc = a ** (s_ + t_) * s0 * s0
            for u in range(1, min(s_, t_) + 1):
                acc += sx * sx * a ** (s_ - u) * a ** (t_ - u)
            cov[i, j] = acc + (sy * sy if i == j else 0.0)
    return st.multivariate_normal(mean, cov).logpdf(y)
