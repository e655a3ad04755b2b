"""Python binding of libsmc2.so (include/smc2.h, include/smc2_kernels.h).

Argument marshalling only: every step of the sampler runs in the HIP library.
torch provides device memory (uint8 buffers) and the current HIP stream; nothing
else is taken from it. Importing works without a GPU; using the library needs the
built ``libsmc2.so`` (``python -m paper_2311_12973_amd.build``) and raises if it is
missing -- there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmc2.so")

OK, E_ARG, E_DEVICE, E_STATE, E_NUMERIC, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
SIR, SEIR, AGE_SEIR, LINGAUSS = 0, 1, 2, 3
OBS_POIS_PREV, OBS_POIS_INC, OBS_NB_INC, OBS_GAUSS = 0, 1, 2, 3
PREC_FP32, PREC_FP64 = 0, 1
PRIOR_UNIFORM, PRIOR_LOGNORMAL, PRIOR_LOGITNORMAL, PRIOR_NORMAL = 0, 1, 2, 3
L_FORWARD, L_GAUSS_OPT = 0, 1
PROP_RW, PROP_MLP, PROP_LANGEVIN, PROP_RW_POP = 0, 1, 2, 3
PF_RS_SYSTEMATIC, PF_RS_MULTINOMIAL = 0, 1
MLP_TRAIN_AUTO, MLP_TRAIN_PER_RUN, MLP_TRAIN_SPLIT = 0, 1, 2
SCHED_AUTO, SCHED_PER_DRAW, SCHED_POOLED = 0, 1, 2
LAUNCH_AUTO, LAUNCH_PERSISTENT, LAUNCH_PER_FILTER = 0, 1, 2
DUMP = dict(phi=0, lp=1, ll=2, logw=3, phi_new=4, lp_new=5, ll_new=6, logw_pre=7, anc=8, mlp_out=9, logq=10,
            mlp_params=11, mlp_frame=12, mlp_state=13, mlp_grad=14, psteps=15, lkfit=16, theta_new=17, score=18,
            score_new=19)
MLP_H = 64
PMCMC_PHI, PMCMC_LL, PMCMC_LL_PROPOSED, PMCMC_ACCEPTED = 0, 1, 2, 3


def mlp_nout(D):
    return D + D * (D + 1) // 2


def mlp_nparams(D):
    P = mlp_nout(D)
    return MLP_H * D + MLP_H + MLP_H * MLP_H + MLP_H + P * MLP_H + P
NFIXED = 32


def record_len(D):
    return 8 + 2 * D + D * D


class Smc2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("smc2 error %d: %s" % (code, msg))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("obs", ctypes.c_int32), ("D", ctypes.c_int32), ("N", ctypes.c_int32),
                ("K", ctypes.c_int32), ("precision", ctypes.c_int32), ("proposal", ctypes.c_int32),
                ("lkernel", ctypes.c_int32), ("pf_always", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("block", ctypes.c_int32), ("schedule", ctypes.c_int32), ("n_pop", ctypes.c_double),
                ("prior", ctypes.POINTER(ctypes.c_double)), ("rw_cov", ctypes.POINTER(ctypes.c_double)),
                ("fixed", ctypes.POINTER(ctypes.c_double)), ("n_fixed", ctypes.c_int32),
                ("tune", ctypes.c_int32), ("persistent", ctypes.c_int32), ("mlp_epochs", ctypes.c_int32),
                ("mlp_batch", ctypes.c_int32), ("mlp_lr", ctypes.c_double), ("pf_resampling", ctypes.c_int32),
                ("mlp_train", ctypes.c_int32), ("lgv_step", ctypes.c_double)]


class Run(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("n_x", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("y", ctypes.POINTER(ctypes.c_int32)), ("y_real", ctypes.POINTER(ctypes.c_double))]


class StepInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("resampled", ctypes.c_int32), ("dead", ctypes.c_int32),
                ("lkernel_fallback", ctypes.c_int32), ("learned", ctypes.c_int32), ("proposal", ctypes.c_int32),
                ("ess", ctypes.c_double), ("log_weight_sum", ctypes.c_double), ("particle_steps", ctypes.c_uint64),
                ("ms_filters", ctypes.c_double), ("ms_outer", ctypes.c_double), ("ms_mlp", ctypes.c_double),
                ("ms_step", ctypes.c_double)]


_lib = None


def lib():
    """Load libsmc2.so; raises when it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname as the system one;
        # loading torch first makes libsmc2.so bind to that runtime, so the library and
        # torch share one HIP runtime (and torch's streams are valid for the library).
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsmc2.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2311_12973_amd.build); no fallback exists")
        L = ctypes.CDLL(LIB_PATH)
        c, P = ctypes, ctypes.POINTER
        vp = c.c_void_p
        L.smc2_workspace_bytes.restype = c.c_size_t
        L.smc2_workspace_bytes.argtypes = [P(Config), c.c_int32, P(Run)]
        L.smc2_init.restype = c.c_int
        L.smc2_init.argtypes = [P(Config), c.c_int32, P(Run), vp, c.c_size_t, vp, P(vp)]
        L.smc2_step.restype = c.c_int
        L.smc2_step.argtypes = [vp]
        L.smc2_records.restype = c.c_int
        L.smc2_records.argtypes = [vp, c.c_int32, P(c.c_double), c.c_size_t, P(c.c_int32)]
        L.smc2_estimate.restype = c.c_int
        L.smc2_estimate.argtypes = [vp, c.c_int32, c.c_int32, P(c.c_double), P(c.c_double)]
        L.smc2_dump.restype = c.c_int
        L.smc2_dump.argtypes = [vp, c.c_int32, c.c_int32, vp, c.c_size_t]
        L.smc2_info.restype = c.c_int
        L.smc2_info.argtypes = [vp, c.c_int32, c.c_int32, P(StepInfo)]
        L.smc2_timing.restype = c.c_int
        L.smc2_timing.argtypes = [vp, P(c.c_double), P(c.c_double), P(c.c_int32)]
        L.smc2_destroy.restype = c.c_int
        L.smc2_destroy.argtypes = [vp]
        L.smc2_last_error.restype = c.c_char_p
        L.smc2_mlp_forward.restype = c.c_int
        L.smc2_mlp_forward.argtypes = [c.c_int32, c.c_int32, vp, vp, vp, vp, vp]
        L.smc2_mlp_grad.restype = c.c_int
        L.smc2_mlp_grad.argtypes = [c.c_int32, c.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.smc2_groups.restype = c.c_int
        L.smc2_groups.argtypes = [vp, c.c_int32, P(c.c_int32), P(c.c_int32), P(c.c_float)]
        L.smc2_last_error.argtypes = [vp]
        L.smc2_philox_batch.restype = c.c_int
        L.smc2_philox_batch.argtypes = [c.c_int32, vp, c.c_uint64, vp, vp]
        L.smc2_binomial_batch.restype = c.c_int
        L.smc2_binomial_batch.argtypes = [c.c_int32, c.c_int32, vp, vp, c.c_uint64, c.c_uint32, c.c_uint32,
                                          c.c_uint32, c.c_uint32, vp, vp]
        L.smc2_resample_batch.restype = c.c_int
        L.smc2_resample_batch.argtypes = [c.c_int32, c.c_int32, vp, vp, vp, vp, vp]
        L.smc2_pf_workspace_bytes.restype = c.c_size_t
        L.smc2_pf_workspace_bytes.argtypes = [P(Config), P(Run)]
        L.smc2_pf_trace.restype = c.c_int
        L.smc2_pf_trace.argtypes = [P(Config), c.c_int32, vp, P(Run), c.c_uint32, vp, vp, vp, vp, c.c_size_t, vp]
        L.smc2_pf_trace_state.restype = c.c_int
        L.smc2_pf_trace_state.argtypes = [P(Config), c.c_int32, vp, P(Run), c.c_uint32, vp, vp, vp, vp, vp, vp,
                                          c.c_size_t, vp]
        L.smc2_pf_loglik.restype = c.c_int
        L.smc2_pf_loglik.argtypes = [P(Config), c.c_int32, vp, P(Run), c.c_uint32, vp, vp, c.c_size_t, vp]
        L.smc2_pf_score.restype = c.c_int
        L.smc2_pf_score.argtypes = [P(Config), c.c_int32, vp, P(Run), c.c_uint32, vp, vp, vp, c.c_size_t, vp]
        L.smc2_pf_loglik_noalloc.restype = c.c_int
        L.smc2_pf_loglik_noalloc.argtypes = [P(Config), c.c_int32, vp, P(Run), c.c_uint32, vp, vp]
        L.smc2_pmcmc_workspace_bytes.restype = c.c_size_t
        L.smc2_pmcmc_workspace_bytes.argtypes = [P(Config), c.c_int32, c.c_int32, P(Run)]
        L.smc2_pmcmc_init.restype = c.c_int
        L.smc2_pmcmc_init.argtypes = [P(Config), c.c_int32, c.c_int32, P(Run), vp, c.c_size_t, vp, P(vp)]
        L.smc2_pmcmc_step.restype = c.c_int
        L.smc2_pmcmc_step.argtypes = [vp, c.c_int32]
        L.smc2_pmcmc_estimate.restype = c.c_int
        L.smc2_pmcmc_estimate.argtypes = [vp, c.c_int32, P(c.c_double), P(c.c_double), P(c.c_double)]
        L.smc2_pmcmc_dump.restype = c.c_int
        L.smc2_pmcmc_dump.argtypes = [vp, c.c_int32, vp, c.c_size_t]
        L.smc2_pmcmc_timing.restype = c.c_int
        L.smc2_pmcmc_timing.argtypes = [vp, P(c.c_double), P(c.c_int32)]
        L.smc2_pmcmc_destroy.restype = c.c_int
        L.smc2_pmcmc_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != OK:
        msg = lib().smc2_last_error(ctx)
        raise Smc2Error(rc, msg.decode() if msg else "")
    return rc


# ------------------------------------------------------------------ device buffers (torch)
def _torch():
    import torch
    return torch


def device_buffer(nbytes, device="cuda"):
    """A 256-byte aligned uint8 device buffer: (tensor, pointer)."""
    t = _torch().empty(int(nbytes) + 256, dtype=_torch().uint8, device=device)
    p = t.data_ptr()
    return t, p + ((-p) % 256)


def to_device(arr, device="cuda"):
    a = np.ascontiguousarray(arr)
    t = _torch().from_numpy(a.view(np.uint8).reshape(-1).copy()).to(device)
    return t, t.data_ptr()


def from_device(t, ptr, dtype, count):
    torch = _torch()
    nbytes = np.dtype(dtype).itemsize * count
    off = ptr - t.data_ptr()
    host = t[off:off + nbytes].cpu().numpy()
    return host.view(dtype).copy()


def current_stream():
    return _torch().cuda.current_stream().cuda_stream


# ------------------------------------------------------------------ configs
class _Keep:
    """Host arrays referenced by a Config / Run array (kept alive with them)."""


def make_config(w, N=None, K=None, precision=None, use_graph=0, block=0, lkernel=None, pf_always=None,
                schedule=0, tune=0, persistent=0, proposal=None):
    keep = _Keep()
    D = int(w["D"])
    keep.prior = np.ascontiguousarray(np.asarray(w["prior"], dtype=np.float64).reshape(D, 3))
    keep.rw = np.ascontiguousarray(np.asarray(w["rw_cov"], dtype=np.float64).reshape(D, D))
    keep.fixed = np.zeros(NFIXED, dtype=np.float64)
    fx = list(w.get("fixed", []))
    keep.fixed[:len(fx)] = fx
    c = Config()
    c.model, c.obs, c.D = int(w["model"]), int(w["obs"]), D
    c.N = int(N if N is not None else w["N"])
    c.K = int(K if K is not None else w["K"])
    c.precision = int(precision if precision is not None else w["prec"])
    c.proposal = int(proposal if proposal is not None else w.get("proposal", PROP_RW))
    c.mlp_epochs = int(w.get("mlp_epochs", 4))
    c.mlp_batch = int(w.get("mlp_batch", 256))
    c.mlp_lr = float(w.get("mlp_lr", 1e-3))
    c.lkernel = int(lkernel if lkernel is not None else w.get("lkernel", L_GAUSS_OPT))
    c.pf_always = int(pf_always if pf_always is not None else w.get("pf_always", 0))
    c.use_graph, c.block, c.schedule = int(use_graph), int(block), int(schedule)
    c.tune, c.persistent = int(tune), int(persistent)
    c.pf_resampling = int(w.get("pf_resampling", PF_RS_SYSTEMATIC))
    c.mlp_train = int(w.get("mlp_train", MLP_TRAIN_AUTO))
    c.lgv_step = float(w.get("lgv_step", 0.0))
    c.n_pop = float(w["n_pop"])
    dp = ctypes.POINTER(ctypes.c_double)
    c.prior = keep.prior.ctypes.data_as(dp)
    c.rw_cov = keep.rw.ctypes.data_as(dp)
    c.fixed = keep.fixed.ctypes.data_as(dp)
    c.n_fixed = len(fx)
    c._keep = keep
    return c


def obs_array(y):
    """Observations as the ABI takes them: float64 reals (the linear-Gaussian model) stay
    float64, counts become int32."""
    a = np.asarray(y)
    return np.ascontiguousarray(a, dtype=np.float64 if np.issubdtype(a.dtype, np.floating) else np.int32)


def make_runs(runs):
    """runs: list of dict(T, nx, seed, y); a floating-point y (the linear-Gaussian model)
    goes to y_real, counts to y."""
    arr = (Run * len(runs))()
    keep = []
    for r, d in enumerate(runs):
        y = obs_array(d["y"])
        keep.append(y)
        arr[r].T = int(d.get("T", y.shape[0]))
        arr[r].n_x = int(d["nx"])
        arr[r].seed = int(d["seed"])
        if y.dtype == np.float64:
            arr[r].y_real = y.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            arr[r].y = y.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    arr._keep = keep
    return arr


# ------------------------------------------------------------------ the sampler
class Sampler:
    """One SMC^2 context (smc2_init / smc2_step / smc2_estimate) on the current HIP stream."""

    def __init__(self, w, runs, device="cuda", **cfg_over):
        self.cfg = make_config(w, **cfg_over)
        self.runs = make_runs(runs)
        self.R = len(runs)
        L = lib()
        nbytes = L.smc2_workspace_bytes(ctypes.byref(self.cfg), self.R, self.runs)
        if nbytes == 0:
            _check(E_ARG)
        self.ws, self.ws_ptr = device_buffer(nbytes, device)
        self.stream = current_stream()
        h = ctypes.c_void_p()
        _check(L.smc2_init(ctypes.byref(self.cfg), self.R, self.runs, ctypes.c_void_p(self.ws_ptr), nbytes,
                           ctypes.c_void_p(self.stream), ctypes.byref(h)))
        self.h = h
        self.D = self.cfg.D
        self.N = self.cfg.N

    def step(self):
        _check(lib().smc2_step(self.h), self.h)

    def records(self, run=0):
        RL = record_len(self.D)
        buf = np.zeros((self.cfg.K, RL))
        kd = ctypes.c_int32()
        _check(lib().smc2_records(self.h, run, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), buf.size,
                                  ctypes.byref(kd)), self.h)
        return buf[:kd.value]

    def estimate(self, run=0, recycled=True):
        mean = np.zeros(self.D)
        cov = np.zeros((self.D, self.D))
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().smc2_estimate(self.h, run, int(recycled), mean.ctypes.data_as(dp), cov.ctypes.data_as(dp)),
               self.h)
        return mean, cov

    def dump(self, what, run=0):
        code = DUMP[what]
        if what in ("phi", "phi_new", "theta_new", "score", "score_new"):
            out = np.zeros((self.N, self.D))
        elif what == "anc":
            out = np.zeros(self.N, dtype=np.int32)
        elif what == "mlp_out":
            out = np.zeros((self.N, mlp_nout(self.D)), dtype=np.float32)
        elif what in ("mlp_params", "mlp_grad"):
            out = np.zeros(mlp_nparams(self.D), dtype=np.float32)
        elif what == "mlp_frame":
            out = np.zeros(self.D + self.D * self.D)
        elif what == "mlp_state":
            out = np.zeros(4)
        elif what == "psteps":
            out = np.zeros(1, dtype=np.uint64)
        elif what == "lkfit":
            out = np.zeros(2 * self.D + 4 * self.D * self.D)
        else:
            out = np.zeros(self.N)
        _check(lib().smc2_dump(self.h, code, run, out.ctypes.data_as(ctypes.c_void_p), out.nbytes), self.h)
        return out

    def info(self, k, run=0):
        """smc2_info of completed iteration k (1-based) as a dict."""
        out = StepInfo()
        _check(lib().smc2_info(self.h, run, int(k), ctypes.byref(out)), self.h)
        return {name: getattr(out, name) for name, _ in StepInfo._fields_}

    def timing(self):
        a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        _check(lib().smc2_timing(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)), self.h)
        return a.value, b.value, n.value

    def groups(self):
        """Launch groups of the particle-filter batch and their configuration."""
        L = lib()
        n = ctypes.c_int32()
        _check(L.smc2_groups(self.h, 0, ctypes.byref(n), None, None), self.h)
        desc = (ctypes.c_int32 * (6 * max(n.value, 1)))()
        ms = (ctypes.c_float * max(n.value, 1))()
        _check(L.smc2_groups(self.h, n.value, ctypes.byref(n), desc, ms), self.h)
        keys = ("block", "schedule", "persistent", "grid", "filters", "lds")
        return [dict(zip(keys, desc[6 * g:6 * g + 6]), tuned_ms=float(ms[g])) for g in range(n.value)]

    def close(self):
        if getattr(self, "h", None):
            lib().smc2_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ kernel-level entry points
def philox_batch(ctr, seed, device="cuda"):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    n = ctr.shape[0]
    tc, pc = to_device(ctr, device)
    to, po = device_buffer(16 * n, device)
    _check(lib().smc2_philox_batch(n, pc, int(seed), po, current_stream()))
    return from_device(to, po, np.uint32, 4 * n).reshape(n, 4)


def binomial_batch(precision, n, p, seed, i=0, k=1, t=1, b=0, device="cuda"):
    n = np.ascontiguousarray(n, dtype=np.int32)
    p = np.ascontiguousarray(p, dtype=np.float64)
    cnt = n.size
    tn, pn = to_device(n, device)
    tp, pp = to_device(p, device)
    to, po = device_buffer(4 * cnt, device)
    _check(lib().smc2_binomial_batch(precision, cnt, pn, pp, int(seed), i, k, t, b, po, current_stream()))
    return from_device(to, po, np.int32, cnt)


def resample_batch(q, x64, device="cuda"):
    q = np.ascontiguousarray(q, dtype=np.uint64)
    if q.ndim == 1:
        q = q[None, :]
    S, n = q.shape
    x64 = np.ascontiguousarray(x64, dtype=np.uint64).reshape(S)
    tq, pq = to_device(q, device)
    tx, px = to_device(x64, device)
    ta, pa = device_buffer(4 * S * n, device)
    tt, pt = device_buffer(4 * S, device)
    _check(lib().smc2_resample_batch(S, n, pq, px, pa, pt, current_stream()))
    return from_device(ta, pa, np.int32, S * n).reshape(S, n), from_device(tt, pt, np.int32, S)


def pf_trace_state(w, theta, y, nx, seed, k, precision=None, block=0, device="cuda", schedule=0, with_anc=False):
    """(ll, inc[n][T], rs[n][T], state[n][T][n_counts][nx]) for the rows of theta, and
    with_anc=True also anc[n][T][nx], the ancestors chosen after each day."""
    cfg = make_config(w, N=max(2, len(theta)), K=1, precision=precision, block=block, schedule=schedule)
    y = obs_array(y)
    runs = make_runs([dict(T=y.shape[0], nx=nx, seed=seed, y=y)])
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    n, T = theta.shape[0], y.shape[0]
    nc = {SIR: 2, SEIR: 3, AGE_SEIR: 12, LINGAUSS: 2}[cfg.model]
    L = lib()
    wsb = L.smc2_pf_workspace_bytes(ctypes.byref(cfg), runs)
    tws, pws = device_buffer(wsb, device)
    tth, pth = to_device(theta, device)
    tll, pll = device_buffer(8 * n, device)
    tinc, pinc = device_buffer(8 * n * T, device)
    trs, prs = device_buffer(4 * n * T, device)
    tst, pst = device_buffer(4 * n * T * nc * nx, device)
    tanc, panc = device_buffer(4 * n * T * nx, device) if with_anc else (None, None)
    _check(L.smc2_pf_trace_state(ctypes.byref(cfg), n, pth, runs, int(k), pll, pinc, prs, pst, panc, pws, wsb,
                                 current_stream()))
    out = (from_device(tll, pll, np.float64, n), from_device(tinc, pinc, np.float64, n * T).reshape(n, T),
           from_device(trs, prs, np.int32, n * T).reshape(n, T),
           from_device(tst, pst, np.int32, n * T * nc * nx).reshape(n, T, nc, nx))
    if with_anc:
        out = out + (from_device(tanc, panc, np.int32, n * T * nx).reshape(n, T, nx),)
    return out


def pf_loglik(w, theta, y, nx, seed, k, precision=None, pf_always=None, block=0, device="cuda", trace=False,
              schedule=0):
    """Particle-filter log-likelihoods for the rows of theta (natural parameters);
    with trace=True also the per-day increments and resampling flags."""
    cfg = make_config(w, N=max(2, len(theta)), K=1, precision=precision, pf_always=pf_always, block=block,
                      schedule=schedule)
    y = obs_array(y)
    runs = make_runs([dict(T=y.shape[0], nx=nx, seed=seed, y=y)])
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    n = theta.shape[0]
    L = lib()
    wsb = L.smc2_pf_workspace_bytes(ctypes.byref(cfg), runs)
    tws, pws = device_buffer(wsb, device)
    tth, pth = to_device(theta, device)
    tll, pll = device_buffer(8 * n, device)
    if not trace:
        _check(L.smc2_pf_loglik(ctypes.byref(cfg), n, pth, runs, int(k), pll, pws, wsb, current_stream()))
        return from_device(tll, pll, np.float64, n)
    T = y.shape[0]
    tinc, pinc = device_buffer(8 * n * T, device)
    trs, prs = device_buffer(4 * n * T, device)
    _check(L.smc2_pf_trace(ctypes.byref(cfg), n, pth, runs, int(k), pll, pinc, prs, pws, wsb, current_stream()))
    return (from_device(tll, pll, np.float64, n), from_device(tinc, pinc, np.float64, n * T).reshape(n, T),
            from_device(trs, prs, np.int32, n * T).reshape(n, T))


def pf_score(w, theta, y, nx, seed, k, precision=None, pf_always=None, block=0, device="cuda", schedule=0):
    """(log-likelihood estimates [n], score estimates [n][D] on the natural parameters)
    for the rows of theta (smc2_pf_score)."""
    cfg = make_config(w, N=max(2, len(theta)), K=1, precision=precision, pf_always=pf_always, block=block,
                      schedule=schedule)
    y = obs_array(y)
    runs = make_runs([dict(T=y.shape[0], nx=nx, seed=seed, y=y)])
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    n, D = theta.shape
    L = lib()
    wsb = L.smc2_pf_workspace_bytes(ctypes.byref(cfg), runs)
    tws, pws = device_buffer(wsb, device)
    tth, pth = to_device(theta, device)
    tll, pll = device_buffer(8 * n, device)
    tsc, psc = device_buffer(8 * n * D, device)
    _check(L.smc2_pf_score(ctypes.byref(cfg), n, pth, runs, int(k), pll, psc, pws, wsb, current_stream()))
    return from_device(tll, pll, np.float64, n), from_device(tsc, psc, np.float64, n * D).reshape(n, D)


def pf_loglik_noalloc(w, theta, y, nx, seed, k, precision=None, pf_always=None, block=0, device="cuda", schedule=0):
    """As pf_loglik through smc2_pf_loglik_noalloc (no workspace: the library stages the
    run in its static device scratch)."""
    cfg = make_config(w, N=max(2, len(theta)), K=1, precision=precision, pf_always=pf_always, block=block,
                      schedule=schedule)
    y = obs_array(y)
    runs = make_runs([dict(T=y.shape[0], nx=nx, seed=seed, y=y)])
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    n = theta.shape[0]
    tth, pth = to_device(theta, device)
    tll, pll = device_buffer(8 * n, device)
    _check(lib().smc2_pf_loglik_noalloc(ctypes.byref(cfg), n, pth, runs, int(k), pll, current_stream()))
    return from_device(tll, pll, np.float64, n)


# ------------------------------------------------------------------ learned proposal, kernel level
def mlp_forward(D, params, frame, phi, device="cuda"):
    """Network outputs (n x P, float32) of rows phi (n x D) on the GPU."""
    phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1, D)
    n = phi.shape[0]
    tp, pp = to_device(np.ascontiguousarray(params, dtype=np.float32), device)
    tf, pf = to_device(np.ascontiguousarray(frame, dtype=np.float64), device)
    tx, px = to_device(phi, device)
    to, po = device_buffer(4 * max(n, 1) * mlp_nout(D), device)
    _check(lib().smc2_mlp_forward(D, n, pp, pf, px, po, current_stream()))
    return from_device(to, po, np.float32, n * mlp_nout(D)).reshape(n, mlp_nout(D))


def mlp_grad(D, params, frame, phi_in, phi_t, w, device="cuda"):
    """(gradient (NP float32), loss) of sum_r w_r NLL(target_r | input_r) on the GPU."""
    phi_in = np.ascontiguousarray(phi_in, dtype=np.float64).reshape(-1, D)
    phi_t = np.ascontiguousarray(phi_t, dtype=np.float64).reshape(-1, D)
    n = phi_in.shape[0]
    bufs = [to_device(np.ascontiguousarray(x, dtype=dt), device) for x, dt in
            ((params, np.float32), (frame, np.float64), (phi_in, np.float64), (phi_t, np.float64), (w, np.float64))]
    tg, pg = device_buffer(4 * mlp_nparams(D), device)
    tl, pl = device_buffer(8, device)
    _check(lib().smc2_mlp_grad(D, n, *[b[1] for b in bufs], pg, pl, current_stream()))
    return from_device(tg, pg, np.float32, mlp_nparams(D)), float(from_device(tl, pl, np.float64, 1)[0])


# ------------------------------------------------------------------ p-MCMC
class PMCMC:
    """Particle marginal Metropolis-Hastings (smc2_pmcmc_*): `chains` independent chains of
    up to `iters` iterations on the current HIP stream, every chain's filter in one launch
    per iteration. Uses the workload's model, observations, prior and random-walk
    covariance; run = dict(T, nx, seed, y)."""

    def __init__(self, w, run, chains, iters, device="cuda", **cfg_over):
        self.cfg = make_config(w, N=2, K=1, **cfg_over)
        self.runs = make_runs([run])
        self.C, self.iters, self.D = int(chains), int(iters), self.cfg.D
        L = lib()
        nbytes = L.smc2_pmcmc_workspace_bytes(ctypes.byref(self.cfg), self.C, self.iters, self.runs)
        if nbytes == 0:
            _check(E_ARG)
        self.ws, self.ws_ptr = device_buffer(nbytes, device)
        h = ctypes.c_void_p()
        _check(L.smc2_pmcmc_init(ctypes.byref(self.cfg), self.C, self.iters, self.runs, ctypes.c_void_p(self.ws_ptr),
                                 nbytes, ctypes.c_void_p(current_stream()), ctypes.byref(h)))
        self.h = h

    def step(self, n=1):
        _check(lib().smc2_pmcmc_step(self.h, int(n)))

    def estimate(self, burn_in):
        """(mean, covariance, acceptance rate) over the states after burn_in iterations."""
        mean = np.zeros(self.D)
        cov = np.zeros((self.D, self.D))
        rate = ctypes.c_double()
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().smc2_pmcmc_estimate(self.h, int(burn_in), mean.ctypes.data_as(dp), cov.ctypes.data_as(dp),
                                         ctypes.byref(rate)))
        return mean, cov, rate.value

    def dump(self, what):
        code = dict(phi=PMCMC_PHI, ll=PMCMC_LL, ll_proposed=PMCMC_LL_PROPOSED, accepted=PMCMC_ACCEPTED)[what]
        C, I, D = self.C, self.iters, self.D
        out = {"phi": lambda: np.zeros((C, I + 1, D)), "ll": lambda: np.zeros((C, I + 1)),
               "ll_proposed": lambda: np.zeros((C, I)), "accepted": lambda: np.zeros((C, I), dtype=np.int32)}[what]()
        _check(lib().smc2_pmcmc_dump(self.h, code, out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def timing(self):
        ms, n = ctypes.c_double(), ctypes.c_int32()
        _check(lib().smc2_pmcmc_timing(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "h", None):
            lib().smc2_pmcmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
