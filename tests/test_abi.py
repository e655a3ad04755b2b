"""The C ABI without a GPU: the library loads, exports every function the headers
declare, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2311_12973_amd as G
from paper_2311_12973_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("smc2.h", "smc2_kernels.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(smc2_[a-z_0-9]+)\s*\(", src, re.M))
    return names


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert {"smc2_init", "smc2_step", "smc2_estimate", "smc2_dump", "smc2_destroy", "smc2_workspace_bytes",
            "smc2_pf_loglik", "smc2_resample_batch", "smc2_binomial_batch", "smc2_philox_batch"} <= names
    L = G.lib()
    for n in sorted(names):
        assert hasattr(L, n), n


def _w():
    return W.preset("seir")


def test_workspace_bytes_and_validation():
    L = G.lib()
    w = _w()
    y = W.observations(w)
    runs = G.make_runs([dict(T=100, nx=512, seed=1, y=y)])
    cfg = G.make_config(w)
    nb = L.smc2_workspace_bytes(ctypes.byref(cfg), 1, runs)
    assert 3 * 1024 * 4 * 8 < nb < 1 << 20  # O(N D) doubles: particles never leave the chip
    bad = [dict(N=1), dict(N=40000), dict(K=0), dict(precision=3), dict(block=96), dict(block=2048),
           dict(schedule=3), dict(schedule=-1), dict(persistent=3), dict(persistent=-1)]
    bad_w = [dict(lgv_step=-0.1), dict(lgv_step=1.5), dict(lgv_step=float("nan"))]
    for over in bad:
        c = G.make_config(w, **over)
        assert L.smc2_workspace_bytes(ctypes.byref(c), 1, runs) == 0, over
    for over in bad_w:
        c = G.make_config(dict(w, **over))
        assert L.smc2_workspace_bytes(ctypes.byref(c), 1, runs) == 0, over
    c = G.make_config(dict(w, D=3, prior=w["prior"][:3], rw_cov=np.eye(3).tolist()))
    assert L.smc2_workspace_bytes(ctypes.byref(c), 1, runs) == 0
    c = G.make_config(dict(w, rw_cov=(-np.eye(4)).tolist()))
    assert L.smc2_workspace_bytes(ctypes.byref(c), 1, runs) == 0
    assert b"positive definite" in L.smc2_last_error(None)
    for r in [dict(T=100, nx=0, seed=1, y=y), dict(T=0, nx=512, seed=1, y=y[:0]), dict(T=100, nx=5000, seed=1, y=y)]:
        assert L.smc2_workspace_bytes(ctypes.byref(cfg), 1, G.make_runs([r])) == 0, r
    # the learned proposal needs sane settings; it runs with either L-kernel
    for over in [dict(mlp_lr=0.0), dict(mlp_epochs=-1)]:
        cm = G.make_config(dict(w, proposal=G.PROP_MLP, **over))
        assert L.smc2_workspace_bytes(ctypes.byref(cm), 1, runs) == 0, over
    cm = G.make_config(dict(w, proposal=G.PROP_MLP))
    assert L.smc2_workspace_bytes(ctypes.byref(cm), 1, runs) > nb  # network state and outputs
    cf = G.make_config(dict(w, proposal=G.PROP_MLP), lkernel=G.L_FORWARD)
    assert L.smc2_workspace_bytes(ctypes.byref(cf), 1, runs) == L.smc2_workspace_bytes(ctypes.byref(cm), 1, runs)
    wa = W.preset("age_seir")
    ya = W.observations(dict(wa, T=10))
    ca = G.make_config(wa, schedule=G.SCHED_POOLED)
    ra = G.make_runs([dict(T=10, nx=256, seed=1, y=ya)])
    assert L.smc2_workspace_bytes(ctypes.byref(ca), 1, ra) == 0
    assert b"pooled" in L.smc2_last_error(None)
    for v in (2, -1):
        c = G.make_config(dict(w, pf_resampling=v))
        assert L.smc2_workspace_bytes(ctypes.byref(c), 1, runs) == 0
        assert b"pf_resampling" in L.smc2_last_error(None)
    c = G.make_config(dict(w, pf_resampling=G.PF_RS_MULTINOMIAL))
    assert L.smc2_workspace_bytes(ctypes.byref(c), 1, runs) == nb
    for v in (3, -1):
        c = G.make_config(dict(w, mlp_train=v))
        assert L.smc2_workspace_bytes(ctypes.byref(c), 1, runs) == 0
        assert b"mlp_train" in L.smc2_last_error(None)
    yneg = y.copy()
    yneg[3] = -1
    assert L.smc2_workspace_bytes(ctypes.byref(cfg), 1, G.make_runs([dict(T=100, nx=512, seed=1, y=yneg)])) == 0


def test_init_rejects_before_device_use():
    L = G.lib()
    w = _w()
    y = W.observations(w)
    runs = G.make_runs([dict(T=100, nx=512, seed=1, y=y)])
    cfg = G.make_config(w)
    h = ctypes.c_void_p()
    # no workspace / too small / misaligned
    assert L.smc2_init(ctypes.byref(cfg), 1, runs, None, 0, None, ctypes.byref(h)) == G.E_ARG
    assert L.smc2_init(ctypes.byref(cfg), 1, runs, ctypes.c_void_p(4096), 16, None, ctypes.byref(h)) == G.E_ARG
    assert L.smc2_init(ctypes.byref(cfg), 1, runs, ctypes.c_void_p(4097), 1 << 30, None, ctypes.byref(h)) == G.E_ARG
    assert h.value is None
    c = G.make_config(dict(w, obs=W.OBS_POIS_PREV))
    assert L.smc2_init(ctypes.byref(c), 1, runs, ctypes.c_void_p(4096), 1 << 30, None,
                       ctypes.byref(h)) == G.E_UNSUPPORTED
    assert L.smc2_step(None) == G.E_ARG
    assert L.smc2_destroy(None) == G.OK


def test_kernel_entry_points_reject_bad_arguments():
    L = G.lib()
    assert L.smc2_resample_batch(1, 0, None, None, None, None, None) == G.E_ARG
    assert L.smc2_resample_batch(1, 5000, None, None, None, None, None) == G.E_ARG
    assert L.smc2_binomial_batch(7, 1, None, None, 0, 0, 1, 1, 0, None, None) == G.E_ARG
    assert L.smc2_philox_batch(-1, None, 0, None, None) == G.E_ARG
    assert L.smc2_mlp_forward(0, 4, None, None, None, None, None) == G.E_ARG
    assert L.smc2_mlp_forward(9, 4, None, None, None, None, None) == G.E_ARG
    assert L.smc2_mlp_forward(4, 4, None, None, None, None, None) == G.E_ARG
    assert L.smc2_mlp_grad(4, 0, None, None, None, None, None, None, None, None) == G.E_ARG
    # the filter entry point checks every argument before its first copy or launch: these
    # stand-in addresses are never dereferenced
    w = _w()
    y = W.observations(w)
    runs = G.make_runs([dict(T=100, nx=512, seed=1, y=y)])
    fake = ctypes.c_void_p(1 << 20)
    ws = L.smc2_pf_workspace_bytes(ctypes.byref(G.make_config(w)), runs)
    for over, msg in [(dict(block=96), b"block"), (dict(schedule=3), b"schedule")]:
        c = G.make_config(w, **over)
        assert L.smc2_pf_loglik(ctypes.byref(c), 4, fake, runs, 1, fake, fake, ws, None) == G.E_ARG, over
        assert msg in L.smc2_last_error(None)
    ra = G.make_runs([dict(T=10, nx=256, seed=1, y=W.observations(dict(W.preset("age_seir"), T=10)))])
    ca = G.make_config(W.preset("age_seir"), schedule=G.SCHED_POOLED)
    assert L.smc2_pf_loglik(ctypes.byref(ca), 4, fake, ra, 1, fake, fake, ws, None) == G.E_ARG
    assert b"pooled" in L.smc2_last_error(None)


def test_pmcmc_entry_points_reject_bad_arguments():
    L = G.lib()
    w = W.preset("paper_sir")
    y = W.observations(w)
    cfg = G.make_config(w, N=2, K=1)
    runs = G.make_runs([dict(T=30, nx=500, seed=1, y=y)])
    nb = L.smc2_pmcmc_workspace_bytes(ctypes.byref(cfg), 64, 160, runs)
    assert nb > 64 * 161 * 2 * 8  # the chains' traces
    for chains, iters in [(0, 10), (40000, 10), (4, -1), (4, 70000)]:
        assert L.smc2_pmcmc_workspace_bytes(ctypes.byref(cfg), chains, iters, runs) == 0
    h = ctypes.c_void_p()
    assert L.smc2_pmcmc_init(ctypes.byref(cfg), 64, 160, runs, None, 0, None, ctypes.byref(h)) == G.E_ARG
    assert L.smc2_pmcmc_init(ctypes.byref(cfg), 64, 160, runs, ctypes.c_void_p(4097), nb, None,
                             ctypes.byref(h)) == G.E_ARG
    bad = G.make_config(dict(w, rw_cov=(-np.eye(2)).tolist()), N=2, K=1)
    assert L.smc2_pmcmc_init(ctypes.byref(bad), 4, 10, runs, ctypes.c_void_p(4096), nb, None,
                             ctypes.byref(h)) == G.E_ARG
    assert b"positive definite" in L.smc2_last_error(None)
    assert h.value is None
    assert L.smc2_pmcmc_step(None, 1) == G.E_ARG
    assert L.smc2_pmcmc_destroy(None) == G.OK


def test_linear_gaussian_model_validation():
    # real observations through y_real; FP64 only; D = 3; per-draw schedule only
    L = G.lib()
    w = W.preset("lingauss")
    y = W.observations(w)
    runs = G.make_runs([dict(T=w["T"], nx=w["nx"], seed=1, y=y)])
    assert runs[0].y_real and not runs[0].y
    cfg = G.make_config(w)
    nb = L.smc2_workspace_bytes(ctypes.byref(cfg), 1, runs)
    assert nb > 0, L.smc2_last_error(None)
    c32 = G.make_config(w, precision=G.PREC_FP32)
    assert L.smc2_workspace_bytes(ctypes.byref(c32), 1, runs) == 0
    assert b"FP64 only" in L.smc2_last_error(None)
    h = ctypes.c_void_p()
    assert L.smc2_init(ctypes.byref(c32), 1, runs, ctypes.c_void_p(4096), 1 << 30, None,
                       ctypes.byref(h)) == G.E_UNSUPPORTED
    for over in [dict(D=2, prior=w["prior"][:2], rw_cov=np.eye(2).tolist()), dict(obs=W.OBS_NB_INC),
                 dict(fixed=[0.0]), dict(fixed=[0.0, -1.0])]:
        c = G.make_config(dict(w, **over))
        assert L.smc2_workspace_bytes(ctypes.byref(c), 1, runs) == 0, over
    cp = G.make_config(w, schedule=G.SCHED_POOLED)
    assert L.smc2_workspace_bytes(ctypes.byref(cp), 1, runs) == 0
    assert b"pooled" in L.smc2_last_error(None)
    bad = y.copy()
    bad[3] = np.nan
    assert L.smc2_workspace_bytes(ctypes.byref(cfg), 1, G.make_runs([dict(T=w["T"], nx=64, seed=1, y=bad)])) == 0
    assert b"non-finite" in L.smc2_last_error(None)
    # counts where reals are expected: no y_real
    rc = G.make_runs([dict(T=w["T"], nx=64, seed=1, y=np.zeros(w["T"], dtype=np.int32))])
    assert L.smc2_workspace_bytes(ctypes.byref(cfg), 1, rc) == 0
    assert b"y_real" in L.smc2_last_error(None)
    fake = ctypes.c_void_p(1 << 20)
    ws = L.smc2_pf_workspace_bytes(ctypes.byref(cfg), runs)
    assert ws >= 256 + 8 * w["T"]
    assert L.smc2_pf_loglik(ctypes.byref(c32), 4, fake, runs, 1, fake, fake, ws, None) == G.E_UNSUPPORTED


def test_score_entry_point_rejects_before_device_use():
    L = G.lib()
    fake = ctypes.c_void_p(1 << 20)
    wa = W.preset("age_seir")
    ra = G.make_runs([dict(T=10, nx=256, seed=1, y=W.observations(dict(wa, T=10)))])
    ca = G.make_config(wa)
    ws = L.smc2_pf_workspace_bytes(ctypes.byref(ca), ra)
    assert L.smc2_pf_score(ctypes.byref(ca), 4, fake, ra, 1, fake, fake, fake, ws, None) == G.E_UNSUPPORTED
    w = _w()
    runs = G.make_runs([dict(T=100, nx=512, seed=1, y=W.observations(w))])
    c = G.make_config(w)
    ws = L.smc2_pf_workspace_bytes(ctypes.byref(c), runs)
    assert L.smc2_pf_score(ctypes.byref(c), 4, fake, runs, 1, fake, None, fake, ws, None) == G.E_ARG
    c3 = G.make_config(dict(w, D=3, prior=w["prior"][:3], rw_cov=np.eye(3).tolist()))
    assert L.smc2_pf_score(ctypes.byref(c3), 4, fake, runs, 1, fake, fake, fake, ws, None) == G.E_ARG
    # the score launch's LDS: SEIR at N_x = 4096 does not fit with five FP64 score columns
    r4 = G.make_runs([dict(T=100, nx=4096, seed=1, y=W.observations(w))])
    assert L.smc2_pf_score(ctypes.byref(c), 4, fake, r4, 1, fake, fake, fake, ws, None) == G.E_ARG


def test_langevin_proposal_validation():
    L = G.lib()
    w = _w()
    runs = G.make_runs([dict(T=100, nx=512, seed=1, y=W.observations(w))])
    c = G.make_config(w, proposal=G.PROP_LANGEVIN)
    nb = L.smc2_workspace_bytes(ctypes.byref(c), 1, runs)
    assert nb > L.smc2_workspace_bytes(ctypes.byref(G.make_config(w)), 1, runs)  # scores and log q
    wa = dict(W.preset("age_seir"), proposal=G.PROP_LANGEVIN)
    ra = G.make_runs([dict(T=10, nx=256, seed=1, y=W.observations(dict(wa, T=10)))])
    assert L.smc2_workspace_bytes(ctypes.byref(G.make_config(wa)), 1, ra) == 0
    assert b"score" in L.smc2_last_error(None)
    assert L.smc2_workspace_bytes(ctypes.byref(G.make_config(w, proposal=4)), 1, runs) == 0


def test_population_random_walk_validation():
    """every model takes it (no score needed); it holds the log q and the covariance
    factors, not the scores"""
    L = G.lib()
    w = _w()
    runs = G.make_runs([dict(T=100, nx=512, seed=1, y=W.observations(w))])
    base = L.smc2_workspace_bytes(ctypes.byref(G.make_config(w)), 1, runs)
    pop = L.smc2_workspace_bytes(ctypes.byref(G.make_config(w, proposal=G.PROP_RW_POP)), 1, runs)
    lgv = L.smc2_workspace_bytes(ctypes.byref(G.make_config(w, proposal=G.PROP_LANGEVIN)), 1, runs)
    assert base < pop < lgv
    wa = dict(W.preset("age_seir"), proposal=G.PROP_RW_POP)
    ra = G.make_runs([dict(T=10, nx=256, seed=1, y=W.observations(dict(wa, T=10)))])
    assert L.smc2_workspace_bytes(ctypes.byref(G.make_config(wa)), 1, ra) > 0
