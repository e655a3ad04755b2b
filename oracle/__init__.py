"""ctypes binding of the CPU reference (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` import this package. The product path (``paper_2311_12973_amd``) never
does: it must fail loudly when its HIP library is missing instead of falling back
here.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build_oracle

DMAX = 8
NFIXED = 32

SIR, SEIR, AGE_SEIR = 0, 1, 2
OBS_POIS_PREV, OBS_POIS_INC, OBS_NB_INC = 0, 1, 2
PREC_FP32, PREC_FP64 = 0, 1
PRIOR_UNIFORM, PRIOR_LOGNORMAL, PRIOR_LOGITNORMAL, PRIOR_NORMAL = 0, 1, 2, 3
L_FORWARD, L_GAUSS_OPT = 0, 1
PROP_RW, PROP_MLP, PROP_LANGEVIN, PROP_RW_POP = 0, 1, 2, 3
RS_SYSTEMATIC, RS_MULTINOMIAL = 0, 1


class Config(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32), ("obs", ctypes.c_int32), ("D", ctypes.c_int32),
        ("prec", ctypes.c_int32), ("pf_always", ctypes.c_int32), ("lkernel", ctypes.c_int32),
        ("proposal", ctypes.c_int32), ("n_fixed", ctypes.c_int32), ("n_pop", ctypes.c_double),
        ("prior", (ctypes.c_double * 3) * DMAX), ("rw_cov", (ctypes.c_double * DMAX) * DMAX),
        ("fixed", ctypes.c_double * NFIXED), ("mlp_epochs", ctypes.c_int32), ("mlp_batch", ctypes.c_int32),
        ("mlp_lr", ctypes.c_double), ("pf_resampling", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("lgv_step", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        _lib = ctypes.CDLL(LIB)
        _declare(_lib)
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _declare(L):
    c = ctypes
    P = c.POINTER
    L.or_philox.argtypes = [P(c.c_uint32), P(c.c_uint32), P(c.c_uint32)]
    L.or_u24.restype = c.c_float
    L.or_u24.argtypes = [c.c_uint32]
    L.or_u53.restype = c.c_double
    L.or_u53.argtypes = [c.c_uint32, c.c_uint32]
    L.or_normal_call.restype = c.c_double
    L.or_normal_call.argtypes = [c.c_uint64, P(c.c_uint32)]
    L.or_binomial.restype = c.c_int32
    L.or_binomial.argtypes = [c.c_int, c.c_int32, c.c_double, c.c_uint64] + [c.c_uint32] * 5
    L.or_binomial_batch.argtypes = [c.c_int, c.c_int32, c.c_double, c.c_uint64] + [c.c_uint32] * 4 + [
        c.c_int, P(c.c_int32)]
    L.or_binomial_many.argtypes = [c.c_int, c.c_int, P(c.c_int32), P(c.c_double), c.c_uint64] + [
        c.c_uint32] * 4 + [P(c.c_int32)]
    L.or_pf_lg.restype = c.c_double
    L.or_pf_lg.argtypes = [c.c_double] * 5 + [P(c.c_double), c.c_int, c.c_int, c.c_uint64, c.c_uint32, c.c_uint32,
                                              c.c_int, c.c_int, P(c.c_double), P(c.c_int32), P(c.c_double),
                                              P(c.c_double)]
    L.or_propose_langevin_one.restype = c.c_double
    L.or_propose_langevin_one.argtypes = [P(Config), P(c.c_double), P(c.c_double), P(c.c_double), c.c_uint64,
                                          c.c_uint32, c.c_int, P(c.c_double)]
    L.or_digamma.restype = c.c_double
    L.or_digamma.argtypes = [c.c_double]
    L.or_resample_multinomial.argtypes = [P(c.c_uint64), c.c_int, c.c_uint64, c.c_uint32, c.c_uint32, P(c.c_int32)]
    L.or_events_get.argtypes = [P(c.c_double)]
    L.or_events_reset.argtypes = []
    L.or_obs_logpmf.restype = c.c_double
    L.or_obs_logpmf.argtypes = [c.c_int, c.c_int32, c.c_int32, c.c_double]
    L.or_resample_trigger.restype = c.c_int
    L.or_resample_trigger.argtypes = [P(c.c_uint64), c.c_int]
    L.or_resample_ancestors.argtypes = [P(c.c_uint64), c.c_int, c.c_uint64, P(c.c_int32)]
    L.or_cholesky.restype = c.c_int
    L.or_cholesky.argtypes = [c.c_int, P(c.c_double), P(c.c_double)]
    L.or_mvn_logpdf_chol.restype = c.c_double
    L.or_mvn_logpdf_chol.argtypes = [c.c_int, P(c.c_double), P(c.c_double), P(c.c_double)]
    L.or_lkernel_fit.restype = c.c_int
    L.or_lkernel_fit.argtypes = [c.c_int, c.c_int] + [P(c.c_double)] * 6
    L.or_lkernel_fit_cov.restype = c.c_int
    L.or_lkernel_fit_cov.argtypes = [c.c_int, c.c_int] + [P(c.c_double)] * 7
    L.or_prior_logpdf.restype = c.c_double
    L.or_prior_logpdf.argtypes = [P(Config), P(c.c_double)]
    L.or_theta_of_phi.argtypes = [P(Config), P(c.c_double), P(c.c_double)]
    L.or_recycle.argtypes = [c.c_int, c.c_int, P(c.c_double), P(c.c_double), P(c.c_double), P(c.c_double)]
    L.or_pf_score.restype = c.c_double
    L.or_pf_score.argtypes = [P(Config), P(c.c_double), P(c.c_int32), c.c_int, c.c_int, c.c_uint64, c.c_uint32,
                              c.c_uint32, P(c.c_double)]
    L.or_pf_loglik.restype = c.c_double
    L.or_pf_loglik.argtypes = [P(Config), P(c.c_double), P(c.c_int32), c.c_int, c.c_int, c.c_uint64,
                               c.c_uint32, c.c_uint32, P(c.c_double), P(c.c_int32)]
    L.or_pf_trace_state.restype = c.c_double
    L.or_pf_trace_state.argtypes = [P(Config), P(c.c_double), P(c.c_int32), c.c_int, c.c_int, c.c_uint64,
                                    c.c_uint32, c.c_uint32, P(c.c_double), P(c.c_int32), P(c.c_int32)]
    L.or_pf_trace_full.restype = c.c_double
    L.or_pf_trace_full.argtypes = [P(Config), P(c.c_double), P(c.c_int32), c.c_int, c.c_int, c.c_uint64,
                                   c.c_uint32, c.c_uint32, P(c.c_double), P(c.c_int32), P(c.c_int32),
                                   P(c.c_int32)]
    L.or_pf_replay.restype = c.c_double
    L.or_pf_replay.argtypes = [P(Config), P(c.c_double), P(c.c_int32), c.c_int, c.c_int, P(c.c_int32),
                               P(c.c_int32), P(c.c_int32), P(c.c_double)]
    L.or_pmcmc_run.restype = c.c_int
    L.or_pmcmc_run.argtypes = [P(Config), P(c.c_int32), c.c_int, c.c_int, c.c_uint64, c.c_int, c.c_int, c.c_int,
                               P(c.c_double), P(c.c_double), P(c.c_int32)]
    L.or_mh_accept.restype = c.c_int
    L.or_mh_accept.argtypes = [c.c_double] * 5
    L.or_prior_draw.argtypes = [P(Config), c.c_int, c.c_uint64, P(c.c_double), P(c.c_double)]
    L.or_propose_rw.argtypes = [P(Config), c.c_int, c.c_uint64, c.c_uint32, P(c.c_double),
                                P(c.c_double), P(c.c_double)]
    L.or_outer_update.restype = c.c_int
    L.or_outer_update.argtypes = [P(Config), c.c_int, c.c_uint32, c.c_uint64] + [P(c.c_double)] * 8 + [
        P(c.c_double), P(c.c_int32), P(c.c_double)]
    L.or_mlp_nout.restype = c.c_int
    L.or_mlp_nout.argtypes = [c.c_int]
    L.or_mlp_nparams.restype = c.c_int
    L.or_mlp_nparams.argtypes = [c.c_int]
    L.or_mlp_init.argtypes = [c.c_int, c.c_uint64, P(c.c_float)]
    L.or_mlp_forward.argtypes = [c.c_int, P(c.c_float), P(c.c_double), c.c_int, P(c.c_double), P(c.c_double),
                                 P(c.c_double)]
    L.or_mlp_nll.restype = c.c_double
    L.or_mlp_nll.argtypes = [c.c_int, P(c.c_double), P(c.c_double), P(c.c_double)]
    L.or_mlp_backward.argtypes = [c.c_int, P(c.c_float), P(c.c_double), P(c.c_double), P(c.c_double),
                                  P(c.c_double), c.c_int, P(c.c_double)]
    L.or_adam_step.argtypes = [c.c_int, P(c.c_float), P(c.c_float), P(c.c_float), P(c.c_double), c.c_int,
                               c.c_double]
    L.or_mlp_perm.argtypes = [c.c_uint64, c.c_uint32, c.c_uint32, c.c_uint32, c.c_int, P(c.c_uint64),
                              P(c.c_uint64)]
    L.or_mlp_frame.argtypes = [c.c_int, c.c_int, P(c.c_double), P(c.c_double), P(c.c_double)]
    L.or_mlp_frame_len.restype = c.c_int
    L.or_mlp_frame_len.argtypes = [c.c_int]
    L.or_mlp_train.restype = c.c_int
    L.or_mlp_train.argtypes = [P(Config), c.c_int, P(c.c_double), P(c.c_double), c.c_uint64, c.c_uint32, c.c_int,
                               c.c_int, c.c_double, P(c.c_float), P(c.c_float), P(c.c_float), P(c.c_int32),
                               P(c.c_double), P(c.c_double), P(c.c_double)]
    L.or_mlp_propose_one.restype = c.c_double
    L.or_mlp_propose_one.argtypes = [c.c_int, P(c.c_double), P(c.c_double), c.c_uint64, c.c_uint32, c.c_int,
                                     P(c.c_double)]
    L.or_smc2_run.restype = c.c_int
    L.or_smc2_run.argtypes = [P(Config), P(c.c_int32), c.c_int, c.c_int, c.c_uint64, c.c_int, c.c_int,
                              c.c_int, P(c.c_double), P(c.c_double), P(c.c_double), P(c.c_double),
                              P(c.c_double), P(c.c_int32)]
    L.or_record_len.restype = c.c_int
    L.or_record_len.argtypes = [c.c_int]


def make_config(model, obs, D, prec, n_pop, prior, rw_cov, fixed=(), lkernel=L_GAUSS_OPT,
                proposal=PROP_RW, pf_always=0, mlp_epochs=4, mlp_batch=256, mlp_lr=1e-3,
                pf_resampling=RS_SYSTEMATIC, lgv_step=0.0):
    cfg = Config()
    cfg.mlp_epochs, cfg.mlp_batch, cfg.mlp_lr = int(mlp_epochs), int(mlp_batch), float(mlp_lr)
    cfg.model, cfg.obs, cfg.D, cfg.prec = model, obs, D, prec
    cfg.pf_always, cfg.lkernel, cfg.proposal = pf_always, lkernel, proposal
    cfg.pf_resampling = int(pf_resampling)
    cfg.lgv_step = float(lgv_step)
    cfg.n_pop = float(n_pop)
    prior = np.asarray(prior, dtype=np.float64).reshape(D, 3)
    rw = np.asarray(rw_cov, dtype=np.float64).reshape(D, D)
    for d in range(D):
        for e in range(3):
            cfg.prior[d][e] = prior[d, e]
        for e in range(D):
            cfg.rw_cov[d][e] = rw[d, e]
    fixed = list(fixed)
    cfg.n_fixed = len(fixed)
    for a, v in enumerate(fixed):
        cfg.fixed[a] = float(v)
    return cfg


def config_from_workload(w, prec=None):
    """Oracle config from a workload description (paper_2311_12973_amd.workloads)."""
    return make_config(w["model"], w["obs"], w["D"], w["prec"] if prec is None else prec, w["n_pop"],
                       w["prior"], w["rw_cov"], w.get("fixed", ()), w.get("lkernel", L_GAUSS_OPT),
                       w.get("proposal", PROP_RW), w.get("pf_always", 0), w.get("mlp_epochs", 4),
                       w.get("mlp_batch", 256), w.get("mlp_lr", 1e-3), w.get("pf_resampling", RS_SYSTEMATIC),
                       w.get("lgv_step", 0.0))


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def u24(x):
    return lib().or_u24(int(x))


def u53(lo, hi):
    return lib().or_u53(int(lo), int(hi))


def normal_call(seed, ctr):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    return lib().or_normal_call(int(seed), _p(c, ctypes.c_uint32))


def binomial(prec, n, p, seed, j, i, k, t, b):
    return lib().or_binomial(prec, int(n), float(p), int(seed), int(j), int(i), int(k), int(t), int(b))


def binomial_batch(prec, n, p, seed, count, i=0, k=1, t=1, b=0):
    out = np.zeros(count, dtype=np.int32)
    lib().or_binomial_batch(prec, int(n), float(p), int(seed), int(i), int(k), int(t), int(b), int(count),
                            _p(out, ctypes.c_int32))
    return out


def binomial_many(prec, n, p, seed, i=0, k=1, t=1, b=0):
    n = np.ascontiguousarray(n, dtype=np.int32)
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(n.size, dtype=np.int32)
    lib().or_binomial_many(prec, n.size, _p(n, ctypes.c_int32), _p(p, ctypes.c_double), int(seed), int(i), int(k),
                           int(t), int(b), _p(out, ctypes.c_int32))
    return out


def obs_logpmf(obs, y, count, r=0.0):
    return lib().or_obs_logpmf(obs, int(y), int(count), float(r))


def resample_trigger(q):
    q = np.ascontiguousarray(q, dtype=np.uint64)
    return bool(lib().or_resample_trigger(_p(q, ctypes.c_uint64), len(q)))


def resample_ancestors(q, x64):
    q = np.ascontiguousarray(q, dtype=np.uint64)
    anc = np.zeros(len(q), dtype=np.int32)
    lib().or_resample_ancestors(_p(q, ctypes.c_uint64), len(q), int(x64), _p(anc, ctypes.c_int32))
    return anc


def cholesky(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros((n, n))
    st = lib().or_cholesky(n, _p(A, ctypes.c_double), _p(L, ctypes.c_double))
    return st, L


def mvn_logpdf_chol(x, mu, L):
    x = np.ascontiguousarray(x, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    L = np.ascontiguousarray(L, dtype=np.float64)
    return lib().or_mvn_logpdf_chol(len(x), _p(x, ctypes.c_double), _p(mu, ctypes.c_double),
                                    _p(L, ctypes.c_double))


def lkernel_fit(phi, phi_new, omega):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    phi_new = np.ascontiguousarray(phi_new, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    N, D = phi.shape
    mu = np.zeros(2 * D)
    A = np.zeros((D, D))
    LS = np.zeros((D, D))
    st = lib().or_lkernel_fit(N, D, _p(phi, ctypes.c_double), _p(phi_new, ctypes.c_double),
                              _p(omega, ctypes.c_double), _p(mu, ctypes.c_double), _p(A, ctypes.c_double),
                              _p(LS, ctypes.c_double))
    return st, mu, A, LS


def lkernel_fit_cov(phi, phi_new, omega):
    """(status, mu[2D], cov[2D][2D]) of the L-kernel fit's weighted moments."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    phi_new = np.ascontiguousarray(phi_new, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    N, D = phi.shape
    mu = np.zeros(2 * D)
    A = np.zeros((D, D))
    LS = np.zeros((D, D))
    cov = np.zeros((2 * D, 2 * D))
    st = lib().or_lkernel_fit_cov(N, D, _p(phi, ctypes.c_double), _p(phi_new, ctypes.c_double),
                                  _p(omega, ctypes.c_double), _p(mu, ctypes.c_double), _p(A, ctypes.c_double),
                                  _p(LS, ctypes.c_double), _p(cov, ctypes.c_double))
    return st, mu, cov


def prior_logpdf(cfg, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    return lib().or_prior_logpdf(ctypes.byref(cfg), _p(phi, ctypes.c_double))


def theta_of_phi(cfg, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    th = np.zeros_like(phi)
    lib().or_theta_of_phi(ctypes.byref(cfg), _p(phi, ctypes.c_double), _p(th, ctypes.c_double))
    return th


def record_len(D):
    return lib().or_record_len(D)


def recycle(rec, D):
    rec = np.ascontiguousarray(rec, dtype=np.float64)
    K = rec.shape[0]
    mean = np.zeros(D)
    cov = np.zeros((D, D))
    c = np.zeros(K)
    lib().or_recycle(K, D, _p(rec, ctypes.c_double), _p(mean, ctypes.c_double), _p(cov, ctypes.c_double),
                     _p(c, ctypes.c_double))
    return mean, cov, c


def pf_loglik(cfg, theta, y, nx, seed, filt, k, trace=False):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.int32)
    T = y.shape[0]
    inc = np.zeros(T) if trace else None
    rs = np.zeros(T, dtype=np.int32) if trace else None
    ll = lib().or_pf_loglik(ctypes.byref(cfg), _p(theta, ctypes.c_double), _p(y, ctypes.c_int32), T, nx,
                            int(seed), int(filt), int(k),
                            _p(inc, ctypes.c_double) if trace else None,
                            _p(rs, ctypes.c_int32) if trace else None)
    return (ll, inc, rs) if trace else ll


def pf_trace_state(cfg, theta, y, nx, seed, filt, k):
    """(ll, inc[T], rs[T], state[T][n_counts][nx]) of one filter."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.int32)
    T = y.shape[0]
    nc = {SIR: 2, SEIR: 3, AGE_SEIR: 12}[cfg.model]
    inc = np.zeros(T)
    rs = np.zeros(T, dtype=np.int32)
    st = np.zeros((T, nc, nx), dtype=np.int32)
    ll = lib().or_pf_trace_state(ctypes.byref(cfg), _p(theta, ctypes.c_double), _p(y, ctypes.c_int32), T, nx,
                                 int(seed), int(filt), int(k), _p(inc, ctypes.c_double), _p(rs, ctypes.c_int32),
                                 _p(st, ctypes.c_int32))
    return ll, inc, rs, st


def pf_trace_full(cfg, theta, y, nx, seed, filt, k):
    """(ll, inc[T], rs[T], state[T][n_counts][nx], anc[T][nx]) of one filter."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.int32)
    T = y.shape[0]
    nc = {SIR: 2, SEIR: 3, AGE_SEIR: 12}[cfg.model]
    inc = np.zeros(T)
    rs = np.zeros(T, dtype=np.int32)
    st = np.zeros((T, nc, nx), dtype=np.int32)
    anc = np.zeros((T, nx), dtype=np.int32)
    ll = lib().or_pf_trace_full(ctypes.byref(cfg), _p(theta, ctypes.c_double), _p(y, ctypes.c_int32), T, nx,
                                int(seed), int(filt), int(k), _p(inc, ctypes.c_double), _p(rs, ctypes.c_int32),
                                _p(st, ctypes.c_int32), _p(anc, ctypes.c_int32))
    return ll, inc, rs, st, anc


def pf_replay(cfg, theta, y, state, anc, rs):
    """FP64 log-likelihood (and per-day increments) of a filter replayed from another
    implementation's integer decisions: state [T][n_counts][nx], anc [T][nx], rs [T]."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.int32)
    state = np.ascontiguousarray(state, dtype=np.int32)
    anc = np.ascontiguousarray(anc, dtype=np.int32)
    rs = np.ascontiguousarray(rs, dtype=np.int32)
    T, nc, nx = state.shape
    inc = np.zeros(T)
    ll = lib().or_pf_replay(ctypes.byref(cfg), _p(theta, ctypes.c_double), _p(y, ctypes.c_int32), T, nx,
                            _p(state, ctypes.c_int32), _p(anc, ctypes.c_int32), _p(rs, ctypes.c_int32),
                            _p(inc, ctypes.c_double))
    return ll, inc


def pmcmc_run(cfg, y, nx, seed, chains, iters, n_threads=0):
    """Particle marginal Metropolis-Hastings: (theta [chains][iters+1][D], ll [chains][iters+1],
    accepted [chains][iters])."""
    y = np.ascontiguousarray(y, dtype=np.int32)
    T = y.shape[0]
    th = np.zeros((chains, iters + 1, cfg.D))
    ll = np.zeros((chains, iters + 1))
    acc = np.zeros((chains, iters), dtype=np.int32)
    st = lib().or_pmcmc_run(ctypes.byref(cfg), _p(y, ctypes.c_int32), T, nx, int(seed), chains, iters, n_threads,
                            _p(th, ctypes.c_double), _p(ll, ctypes.c_double), _p(acc, ctypes.c_int32))
    assert st == 0
    return th, ll, acc


def mh_accept(lp, ll, lp_new, ll_new, u):
    return bool(lib().or_mh_accept(lp, ll, lp_new, ll_new, u))


def prior_draw(cfg, N, seed):
    phi = np.zeros((N, cfg.D))
    lp = np.zeros(N)
    lib().or_prior_draw(ctypes.byref(cfg), N, int(seed), _p(phi, ctypes.c_double), _p(lp, ctypes.c_double))
    return phi, lp


def propose_rw(cfg, seed, k, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    N = phi.shape[0]
    phi_new = np.zeros_like(phi)
    lp_new = np.zeros(N)
    lib().or_propose_rw(ctypes.byref(cfg), N, int(seed), int(k), _p(phi, ctypes.c_double),
                        _p(phi_new, ctypes.c_double), _p(lp_new, ctypes.c_double))
    return phi_new, lp_new


def outer_update(cfg, k, seed, state, phi_new, lp_new, ll_new, logq=None):
    """state = dict(phi, lp, ll, logw) (updated in place); logq: log q(phi_new | phi) of a
    learned proposal (None: the random walk). Returns (status, logw_pre, anc, rec)."""
    N = phi_new.shape[0]
    for key in ("phi", "lp", "ll", "logw"):
        state[key] = np.ascontiguousarray(state[key], dtype=np.float64)
    phi_new = np.ascontiguousarray(phi_new, dtype=np.float64)
    lp_new = np.ascontiguousarray(lp_new, dtype=np.float64)
    ll_new = np.ascontiguousarray(ll_new, dtype=np.float64)
    if logq is not None:
        logq = np.ascontiguousarray(logq, dtype=np.float64)
    logw_pre = np.zeros(N)
    anc = np.zeros(N, dtype=np.int32)
    rec = np.zeros(record_len(cfg.D))
    d = ctypes.c_double
    st = lib().or_outer_update(ctypes.byref(cfg), N, int(k), int(seed), _p(state["phi"], d), _p(state["lp"], d),
                               _p(state["ll"], d), _p(state["logw"], d), _p(phi_new, d), _p(lp_new, d),
                               _p(ll_new, d), _p(logq, d) if logq is not None else None, _p(logw_pre, d),
                               _p(anc, ctypes.c_int32), _p(rec, d))
    return st, logw_pre, anc, rec


def resample_multinomial(q, seed, filt, kt):
    q = np.ascontiguousarray(q, dtype=np.uint64)
    anc = np.zeros(q.size, dtype=np.int32)
    lib().or_resample_multinomial(_p(q, ctypes.c_uint64), q.size, int(seed), int(filt), int(kt), _p(anc, ctypes.c_int32))
    return anc


def pf_lg(phi, sq, sr, m0, s0, y, nx, seed, filt=0, pf_always=0, trace=False, resampling=RS_SYSTEMATIC, k=0,
          states=False, score=False):
    """Log of the particle filter's likelihood estimate on the scalar linear-Gaussian
    model x_t = phi x_{t-1} + sq e_t, y_t = x_t + sr d_t, x_0 ~ N(m0, s0^2), on the
    streams of iteration k. trace: also the per-day increments and resampling flags;
    states: also the states of each day before resampling (T x nx); score: also the
    estimate of d log p(y) / d(phi, sq, sr)."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    T = y.shape[0]
    inc = np.zeros(T) if trace else None
    rs = np.zeros(T, dtype=np.int32) if trace else None
    xs = np.zeros((T, nx)) if states else None
    sc = np.zeros(3) if score else None
    ll = lib().or_pf_lg(phi, sq, sr, m0, s0, _p(y, ctypes.c_double), T, nx, int(seed), int(filt), int(k),
                        int(pf_always), int(resampling), _p(inc, ctypes.c_double) if trace else None,
                        _p(rs, ctypes.c_int32) if trace else None, _p(xs, ctypes.c_double) if states else None,
                        _p(sc, ctypes.c_double) if score else None)
    out = (ll,) + ((inc, rs) if trace else ()) + ((xs,) if states else ()) + ((sc,) if score else ())
    return out if len(out) > 1 else ll


def pf_score(cfg, theta, y, nx, seed, filt, k):
    """(log-likelihood estimate, score estimate on the natural parameters) of one
    filter (SIR and SEIR)."""
    y = np.ascontiguousarray(y, dtype=np.int32)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    sc = np.zeros(cfg.D)
    ll = lib().or_pf_score(ctypes.byref(cfg), _p(th, ctypes.c_double), _p(y, ctypes.c_int32), y.shape[0], nx,
                           int(seed), int(filt), int(k), _p(sc, ctypes.c_double))
    return ll, sc


def propose_langevin(cfg, phi, s_theta, seed, k, i):
    """(phi_new, log q(phi_new | phi)) of the truncated Langevin proposal of sample i."""
    D = cfg.D
    C = np.array([[cfg.rw_cov[a][c] for c in range(D)] for a in range(D)])
    L = np.ascontiguousarray(np.linalg.cholesky(C))
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    st = np.ascontiguousarray(s_theta, dtype=np.float64)
    out = np.zeros(D)
    lq = lib().or_propose_langevin_one(ctypes.byref(cfg), _p(L, ctypes.c_double), _p(phi, ctypes.c_double),
                                       _p(st, ctypes.c_double), int(seed), int(k), int(i), _p(out, ctypes.c_double))
    return out, lq


def digamma(x):
    return lib().or_digamma(float(x))


# event counters of the particle filter (order of the OR_EV_* enumeration)
EVENTS = ("pstep", "draw", "philox", "inv", "inv_iter", "btrs", "attempt", "final", "t64", "rs_particle")


def events_reset():
    lib().or_events_reset()


def events_get():
    out = np.zeros(len(EVENTS))
    lib().or_events_get(_p(out, ctypes.c_double))
    return dict(zip(EVENTS, out))


def smc2_run(cfg, y, nx, seed, N, K, n_threads=0, dumps=False):
    y = np.ascontiguousarray(y, dtype=np.int32)
    T = y.shape[0]
    D = cfg.D
    rec = np.zeros((K, record_len(D)))
    out = {}
    d = ctypes.c_double
    if dumps:
        out = dict(phi=np.zeros((K, N, D)), ll=np.zeros((K, N)), lp=np.zeros((K, N)), logw=np.zeros((K, N)),
                   anc=np.zeros((K, N), dtype=np.int32))
    st = lib().or_smc2_run(ctypes.byref(cfg), _p(y, ctypes.c_int32), T, nx, int(seed), N, K, n_threads,
                           _p(rec, d),
                           _p(out["phi"], d) if dumps else None, _p(out["ll"], d) if dumps else None,
                           _p(out["lp"], d) if dumps else None, _p(out["logw"], d) if dumps else None,
                           _p(out["anc"], ctypes.c_int32) if dumps else None)
    out["rec"] = rec
    out["status"] = st
    return out


# ------------------------------------------------------------------ learned proposal
MLP_H = 64


def mlp_nout(D):
    return lib().or_mlp_nout(D)


def mlp_nparams(D):
    return lib().or_mlp_nparams(D)


def mlp_init(D, seed):
    w = np.zeros(mlp_nparams(D), dtype=np.float32)
    lib().or_mlp_init(D, int(seed), _p(w, ctypes.c_float))
    return w


def mlp_forward(D, w, u, bf16=True):
    """Outputs o[P] and the hidden activations (h1, h2) of one input row u[D]."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    u = np.ascontiguousarray(u, dtype=np.float64)
    h1, h2, o = np.zeros(MLP_H), np.zeros(MLP_H), np.zeros(mlp_nout(D))
    d = ctypes.c_double
    lib().or_mlp_forward(D, _p(w, ctypes.c_float), _p(u, d), int(bf16), _p(h1, d), _p(h2, d), _p(o, d))
    return o, h1, h2


def mlp_nll(D, o, ut, grad=False):
    o = np.ascontiguousarray(o, dtype=np.float64)
    ut = np.ascontiguousarray(ut, dtype=np.float64)
    g = np.zeros(len(o)) if grad else None
    v = lib().or_mlp_nll(D, _p(o, ctypes.c_double), _p(ut, ctypes.c_double), _p(g, ctypes.c_double) if grad else None)
    return (v, g) if grad else v


def mlp_backward(D, w, u, h1, h2, go, bf16=True):
    """Parameter gradient of one row given d loss / d o."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (u, h1, h2, go)]
    g = np.zeros(mlp_nparams(D))
    d = ctypes.c_double
    lib().or_mlp_backward(D, _p(w, ctypes.c_float), *[_p(x, d) for x in arr], int(bf16), _p(g, d))
    return g


def adam_step(p, m, v, g, t, lr):
    """In place on float32 p, m, v."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().or_adam_step(len(p), _p(p, ctypes.c_float), _p(m, ctypes.c_float), _p(v, ctypes.c_float),
                       _p(g, ctypes.c_double), int(t), float(lr))


def mlp_perm(seed, k, e, which, N):
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    lib().or_mlp_perm(int(seed), int(k), int(e), int(which), int(N), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def mlp_frame(phi, wn):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    wn = np.ascontiguousarray(wn, dtype=np.float64)
    N, D = phi.shape
    fr = np.zeros(D + D * D)
    lib().or_mlp_frame(N, D, _p(phi, ctypes.c_double), _p(wn, ctypes.c_double), _p(fr, ctypes.c_double))
    return fr


def mlp_train(cfg, phi, logw, seed, k, params, adam_m, adam_v, adam_t, epochs=None, batch=None, lr=None):
    """One iteration's training (in place on params, adam_m, adam_v). Returns
    (use_mlp, adam_t, frame, nll_mlp, nll_rw)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    logw = np.ascontiguousarray(logw, dtype=np.float64)
    N, D = phi.shape
    t = ctypes.c_int32(adam_t)
    fr = np.zeros(D + D * D)
    nm, nr = ctypes.c_double(), ctypes.c_double()
    use = lib().or_mlp_train(ctypes.byref(cfg), N, _p(phi, ctypes.c_double), _p(logw, ctypes.c_double), int(seed),
                             int(k), cfg.mlp_epochs if epochs is None else epochs,
                             cfg.mlp_batch if batch is None else batch, cfg.mlp_lr if lr is None else lr,
                             _p(params, ctypes.c_float), _p(adam_m, ctypes.c_float), _p(adam_v, ctypes.c_float),
                             ctypes.byref(t), _p(fr, ctypes.c_double), ctypes.byref(nm), ctypes.byref(nr))
    return use, t.value, fr, nm.value, nr.value


def mlp_propose_one(D, frame, o, seed, k, i):
    frame = np.ascontiguousarray(frame, dtype=np.float64)
    o = np.ascontiguousarray(o, dtype=np.float64)
    phn = np.zeros(D)
    lq = lib().or_mlp_propose_one(D, _p(frame, ctypes.c_double), _p(o, ctypes.c_double), int(seed), int(k), int(i),
                                  _p(phn, ctypes.c_double))
    return phn, lq
