"""Seeded synthetic workloads: configuration presets and simulated observations.

This module is the only code the GPU path and the CPU reference have in common: it
draws the synthetic observation series that both consume (with numpy's own
generator, not the sampler's Philox streams) and holds the preset shapes. It
contains none of the sampler's arithmetic.

The paper measures on simulated SIR data it does not print (Sec. V-A/V-B); every
preset below therefore simulates its own data from a stated seed, at the paper's
shape (``paper_sir``) or at larger epidemic shapes. The model constants and
observation models of each preset are in ``preset``'s table below.
"""
import math

import numpy as np

SIR, SEIR, AGE_SEIR, LINGAUSS = 0, 1, 2, 3
OBS_POIS_PREV, OBS_POIS_INC, OBS_NB_INC, OBS_GAUSS = 0, 1, 2, 3
PREC_FP32, PREC_FP64 = 0, 1
PRIOR_UNIFORM, PRIOR_LOGNORMAL, PRIOR_LOGITNORMAL, PRIOR_NORMAL = 0, 1, 2, 3
L_FORWARD, L_GAUSS_OPT = 0, 1
PROP_RW, PROP_MLP, PROP_LANGEVIN, PROP_RW_POP = 0, 1, 2, 3


def n_obs(model):
    return 4 if model == AGE_SEIR else 1


def _logit(x):
    return math.log(x / (1.0 - x))


def simulate(model, obs, n_pop, theta, T, seed, fixed=(), min_frac=0.01, max_tries=64):
    """Simulate y_{1:T} (int32, shape (T, n_obs)) from the chain-binomial model.

    Redraws with seed+1, seed+2, ... until the total observed count reaches
    ``min_frac`` of the population (an epidemic that took off). The linear-Gaussian
    model gives float64 observations of shape (T,).
    """
    if model == LINGAUSS:
        return _simulate_lg(np.random.Generator(np.random.PCG64(seed)), theta, T, fixed)
    for attempt in range(max_tries):
        rng = np.random.Generator(np.random.PCG64(seed + attempt))
        y = _simulate_once(rng, model, obs, n_pop, theta, T, fixed)
        if y.sum() >= min_frac * n_pop or min_frac <= 0:
            return y
    return y


def _nb(rng, mu, r):
    mu = np.asarray(mu, dtype=np.float64)
    out = np.zeros(mu.shape, dtype=np.int64)
    pos = mu > 0
    if np.any(pos):
        out[pos] = rng.negative_binomial(r, r / (r + mu[pos]))
    return out


def _simulate_once(rng, model, obs, n_pop, th, T, fixed):
    y = np.zeros((T, n_obs(model)), dtype=np.int32)
    if model == SIR:
        beta, gamma = th[0], th[1]
        I = int(fixed[0])
        S = int(n_pop) - I
        for t in range(T):
            nsi = rng.binomial(S, 1.0 - math.exp(-beta * I / n_pop))
            nir = rng.binomial(I, 1.0 - math.exp(-gamma))
            S, I = S - nsi, I + nsi - nir
            lam = I if obs == OBS_POIS_PREV else nsi
            y[t, 0] = rng.poisson(lam) if lam > 0 else 0
    elif model == SEIR:
        beta, sigma, gamma, iota = th[0], th[1], th[2], th[3]
        r = th[4] if len(th) >= 5 else fixed[0]
        I = max(1, int(math.floor(iota * n_pop + 0.5)))
        S, E = int(n_pop) - I, 0
        for t in range(T):
            nse = rng.binomial(S, 1.0 - math.exp(-beta * I / n_pop))
            nei = rng.binomial(E, 1.0 - math.exp(-sigma))
            nir = rng.binomial(I, 1.0 - math.exp(-gamma))
            S, E, I = S - nse, E + nse - nei, I + nei - nir
            y[t, 0] = _nb(rng, [nei], r)[0]
    else:
        beta, sigma, gamma, iota, r = th[0], th[1], th[2], th[3], th[4]
        s = np.array([1.0, th[5], th[6], th[7]])
        C = np.asarray(fixed[:16], dtype=np.float64).reshape(4, 4)
        Ng = np.floor(np.asarray(fixed[16:20]) * n_pop + 0.5).astype(np.int64)
        I = np.maximum(1, np.floor(iota * Ng + 0.5)).astype(np.int64)
        S, E = Ng - I, np.zeros(4, dtype=np.int64)
        for t in range(T):
            lam = beta * s * (C @ (I / Ng))
            nse = rng.binomial(S, 1.0 - np.exp(-lam))
            nei = rng.binomial(E, 1.0 - math.exp(-sigma))
            nir = rng.binomial(I, 1.0 - math.exp(-gamma))
            S, E, I = S - nse, E + nse - nei, I + nei - nir
            y[t, :] = _nb(rng, nei, r)
    return y


def _simulate_lg(rng, th, T, fixed):
    a, sx, sy = th[0], th[1], th[2]
    x = fixed[0] + fixed[1] * rng.standard_normal()
    y = np.empty(T)
    for t in range(T):
        x = a * x + sx * rng.standard_normal()
        y[t] = x + sy * rng.standard_normal()
    return y


def contact_matrix(seed=5):
    """4x4 contact matrix: Dirichlet(1,1,1,1) rows from a fixed seed, scaled to spectral radius 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    C = rng.dirichlet(np.ones(4), size=4)
    return C / np.max(np.abs(np.linalg.eigvals(C)))


def _lognormal_prior(medians, sd):
    return [[PRIOR_LOGNORMAL, math.log(m), sd] for m in medians]


def preset(name, **over):
    """Workload description (dict) for one of the named shapes.

    paper_sir   the paper's SIR experiment shape (Sec. V-A/V-B), synthetic data
    sir_fp64    SIR, N_pop 1e4, Poisson(new cases), T=50, N=64, Nx=64, K=5, FP64
    seir        SEIR, N_pop 1e6, NB(new cases, r=10), T=100, N=1024, Nx=512, K=10, FP32
    seir_batched  256 SEIR runs, uneven T in [30,200] and Nx in {128,...,1024}, N=256
    seir_learned  SEIR with r estimated (D=5), T=150, N=4096, Nx=1024, K=20, MLP proposal
    age_seir    4-group SEIR, T=365, D=8, N=16384, Nx=2048, K=30
    lingauss    scalar linear-Gaussian model (closed-form likelihood), T=100, D=3,
                N=1024, Nx=256, K=10, FP64
    """
    if name == "paper_sir":
        w = dict(model=SIR, obs=OBS_POIS_PREV, D=2, prec=PREC_FP64, n_pop=1e4, fixed=[3],
                 truth=[0.85, 0.20], prior=[[PRIOR_UNIFORM, 0.0, 1.0]] * 2,
                 rw_cov=(0.1 * np.eye(2)).tolist(), T=30, N=1024, nx=500, K=10, data_seed=2311, seed=1)
    elif name == "sir_fp64":
        w = dict(model=SIR, obs=OBS_POIS_INC, D=2, prec=PREC_FP64, n_pop=1e4, fixed=[3],
                 truth=[0.3, 0.1], prior=_lognormal_prior([0.25, 0.1], 0.5),
                 rw_cov=(0.01 * np.eye(2)).tolist(), T=50, N=64, nx=64, K=5, data_seed=1, seed=1)
    elif name == "seir":
        w = dict(model=SEIR, obs=OBS_NB_INC, D=4, prec=PREC_FP32, n_pop=1e6, fixed=[10.0],
                 truth=[0.5, 0.25, 0.2, 2e-5],
                 prior=_lognormal_prior([0.4, 0.2, 0.15], 0.5) + [[PRIOR_LOGITNORMAL, _logit(1e-5), 1.0]],
                 rw_cov=(0.01 * np.eye(4)).tolist(), T=100, N=1024, nx=512, K=10, data_seed=2, seed=1)
    elif name == "seir_batched":
        w = preset("seir")
        w.update(N=256, runs=256, T=None, nx=None, data_seed=None)
    elif name == "seir_learned":
        w = preset("seir")
        w.update(D=5, fixed=[], truth=[0.5, 0.25, 0.2, 2e-5, 10.0],
                 prior=w["prior"] + [[PRIOR_LOGNORMAL, math.log(10.0), 0.5]],
                 rw_cov=(0.01 * np.eye(5)).tolist(), T=150, N=4096, nx=1024, K=20, data_seed=4,
                 proposal=PROP_MLP)
    elif name == "age_seir":
        C = contact_matrix(5)
        w = dict(model=AGE_SEIR, obs=OBS_NB_INC, D=8, prec=PREC_FP32, n_pop=1e6,
                 fixed=C.ravel().tolist() + [0.25] * 4,
                 truth=[0.6, 0.25, 0.2, 2e-5, 10.0, 0.8, 1.2, 0.6],
                 prior=_lognormal_prior([0.4, 0.2, 0.15], 0.5) + [[PRIOR_LOGITNORMAL, _logit(1e-5), 1.0]]
                 + _lognormal_prior([10.0], 0.5) + [[PRIOR_LOGNORMAL, 0.0, 0.5]] * 3,
                 rw_cov=(0.01 * np.eye(8)).tolist(), T=365, N=16384, nx=2048, K=30, data_seed=5, seed=1,
                 proposal=PROP_MLP)
    elif name == "lingauss":
        w = dict(model=LINGAUSS, obs=OBS_GAUSS, D=3, prec=PREC_FP64, n_pop=1.0, fixed=[0.0, 1.0],
                 truth=[0.8, 0.6, 1.0],
                 prior=[[PRIOR_NORMAL, 0.5, 0.4]] + _lognormal_prior([0.5, 0.8], 0.5),
                 rw_cov=(0.01 * np.eye(3)).tolist(), T=100, N=1024, nx=256, K=10, data_seed=8, seed=1)
    else:
        raise KeyError(name)
    w.setdefault("lkernel", L_GAUSS_OPT)
    w.setdefault("proposal", PROP_RW)
    w.setdefault("pf_always", 0)
    w["name"] = name
    w.update(over)
    return w


def observations(w):
    """Simulated y for a single-run workload (int32, (T, n_obs))."""
    return simulate(w["model"], w["obs"], w["n_pop"], w["truth"], w["T"], w["data_seed"], w.get("fixed", ()))


def batched_runs(w, n_runs=None, seed0=1):
    """Per-run (T_r, nx_r, seed_r, y_r) for the batched shape: T_r ~ U{30..200},
    nx_r ~ U{128, 256, 512, 1024}, data simulated at the workload's truth from seed r."""
    n_runs = n_runs or w["runs"]
    runs = []
    for r in range(seed0, seed0 + n_runs):
        rng = np.random.Generator(np.random.PCG64(100000 + r))
        T = int(rng.integers(30, 201))
        nx = int(rng.choice([128, 256, 512, 1024]))
        y = simulate(w["model"], w["obs"], w["n_pop"], w["truth"], T, 7000 + r, w.get("fixed", ()))
        runs.append(dict(T=T, nx=nx, seed=r, y=y))
    return runs
