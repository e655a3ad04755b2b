"""Property test of the C ABI's host-side validation, without a GPU: random configurations
and run descriptions, most of them invalid, go through the sizing calls that validate
(smc2_workspace_bytes, smc2_pmcmc_workspace_bytes) and the filter entry points' size
(smc2_pf_workspace_bytes). None may crash; a rejection (0 bytes) leaves a message; and
whatever is accepted satisfies the limits the headers state (sample and iteration
counts, dimensions fixed by the model, series lengths, particle counts, precision,
proposal, workgroup size, schedule, population size, observations)."""
import ctypes

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import paper_2311_12973_amd as G

MODEL_D = {0: (2,), 1: (4, 5), 2: (8,), 3: (3,)}
MODEL_OBS = {0: (0, 1), 1: (2,), 2: (2,), 3: (3,)}


@st.composite
def case(draw):
    model = draw(st.sampled_from([-1, 0, 1, 2, 3, 7]))
    D = draw(st.sampled_from([0, 1, 2, 3, 4, 5, 8, 9]))
    c = dict(
        model=model, D=D,
        obs=draw(st.sampled_from([-1, 0, 1, 2, 3, 4])),
        N=draw(st.sampled_from([-5, 0, 1, 2, 3, 1000, 32768, 32769])),
        K=draw(st.sampled_from([-1, 0, 1, 10, 65535, 65536])),
        precision=draw(st.sampled_from([-1, 0, 1, 2])),
        proposal=draw(st.sampled_from([-1, 0, 1, 2, 3, 4])),
        lkernel=draw(st.sampled_from([-1, 0, 1, 2])),
        pf_always=draw(st.sampled_from([0, 1])),
        block=draw(st.sampled_from([-64, 0, 64, 96, 256, 1024, 2048])),
        schedule=draw(st.sampled_from([-1, 0, 1, 2, 3])),
        n_pop=draw(st.sampled_from([-1.0, 0.0, 0.5, 1e4, 1e6, 2.0 ** 24, 2.0 ** 25, float("nan"), float("inf")])),
        pf_resampling=draw(st.sampled_from([-1, 0, 1, 2])),
        mlp_epochs=draw(st.sampled_from([-1, 0, 4, 1001])),
        mlp_batch=draw(st.sampled_from([-1, 0, 256])),
        mlp_lr=draw(st.sampled_from([0.0, 1e-3, 1.5])),
        mlp_train=draw(st.sampled_from([-1, 0, 1, 2, 3])),
    )
    nd = max(D, 1)
    fam = draw(st.lists(st.sampled_from([-1, 0, 1, 2, 3, 4]), min_size=nd, max_size=nd))
    b = draw(st.lists(st.sampled_from([-1.0, 0.0, 0.5, 1.0, float("nan")]), min_size=nd, max_size=nd))
    c["prior"] = [[f, -0.5, bb] for f, bb in zip(fam, b)]
    scale = draw(st.sampled_from([0.01, -0.01, 0.0, float("nan")]))
    c["rw_cov"] = (scale * np.eye(nd)).tolist()
    c["n_fixed"] = draw(st.sampled_from([0, 1, 2, 20, 32, 33]))
    c["fixed"] = [draw(st.sampled_from([0.0, 3.0, 0.25, -1.0])) for _ in range(max(c["n_fixed"], 1))]
    runs = []
    for _ in range(draw(st.sampled_from([1, 2]))):
        T = draw(st.sampled_from([-1, 0, 1, 30, 1024, 1025]))
        runs.append(dict(T=T, n_x=draw(st.sampled_from([-1, 0, 1, 64, 2048, 2049, 4096, 4097])),
                         ymin=draw(st.sampled_from([-1, 0, 0, 0])), yreal_bad=draw(st.booleans())))
    c["runs"] = runs
    return c


def _build(c):
    keep = []
    cfg = G.Config()
    for k in ("model", "obs", "D", "N", "K", "precision", "proposal", "lkernel", "pf_always", "block", "schedule",
              "n_fixed", "mlp_epochs", "mlp_batch", "mlp_train", "pf_resampling"):
        setattr(cfg, k, int(c[k]))
    cfg.n_pop, cfg.mlp_lr = float(c["n_pop"]), float(c["mlp_lr"])
    dp = ctypes.POINTER(ctypes.c_double)
    for k in ("prior", "rw_cov", "fixed"):
        a = np.ascontiguousarray(np.asarray(c[k], dtype=np.float64).ravel())
        keep.append(a)
        setattr(cfg, k, a.ctypes.data_as(dp))
    runs = (G.Run * len(c["runs"]))()
    for i, r in enumerate(c["runs"]):
        n = max(r["T"], 1)
        y = np.full(n * 4, 5, dtype=np.int32)
        y[0] = r["ymin"] if r["ymin"] < 0 else y[0]
        yr = np.linspace(-1.0, 1.0, n)
        if r["yreal_bad"]:
            yr[-1] = np.nan
        keep += [y, yr]
        runs[i].T, runs[i].n_x, runs[i].seed = r["T"], r["n_x"], 1
        runs[i].y = y.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        runs[i].y_real = yr.ctypes.data_as(dp)
    return cfg, runs, keep


def _valid_common(c):
    """what the headers state for every accepted configuration"""
    m = c["model"]
    if m not in MODEL_D or c["D"] not in MODEL_D[m] or c["obs"] not in MODEL_OBS[m]:
        return False
    if c["precision"] not in (0, 1) or (m == 3 and c["precision"] != 1):
        return False
    if not (c["block"] == 0 or (64 <= c["block"] <= 1024 and c["block"] % 64 == 0)):
        return False
    if c["schedule"] not in (0, 1, 2) or c["pf_resampling"] not in (0, 1):
        return False
    if m != 3 and not (1 <= c["n_pop"] <= 2 ** 24 and float(c["n_pop"]).is_integer()):
        return False
    for r in c["runs"]:
        if not (1 <= r["T"] <= 1024 and 1 <= r["n_x"] <= (2048 if m == 2 else 4096)):
            return False
        if (m == 3 and r["yreal_bad"]) or (m != 3 and r["ymin"] < 0):
            return False
    return True


@settings(max_examples=400, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(case())
def test_sampler_validation_never_crashes_and_accepts_only_what_the_header_allows(c):
    L = G.lib()
    cfg, runs, keep = _build(c)
    nb = L.smc2_workspace_bytes(ctypes.byref(cfg), len(c["runs"]), runs)
    if nb == 0:
        assert L.smc2_last_error(None), c
        return
    assert _valid_common(c), c
    assert 2 <= c["N"] <= 32768 and 1 <= c["K"] <= 65535, c
    assert c["proposal"] in (0, 1, 2, 3) and c["lkernel"] in (0, 1), c
    if c["proposal"] == 2:
        assert c["model"] in (0, 1, 3), c
    if c["proposal"] == 1:
        assert 0 <= c["mlp_epochs"] <= 1000 and 0 < c["mlp_lr"] < 1 and c["mlp_batch"] >= 0, c
    assert nb >= 8 * c["N"] * c["D"], c


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(case())
def test_kernel_and_pmcmc_validation_never_crash(c):
    """smc2_pf_workspace_bytes is a size only (the filter entry points validate when
    called): positive for any T >= 1, 0 with a message otherwise. The p-MCMC sizing
    validates like the sampler's."""
    L = G.lib()
    cfg, runs, keep = _build(c)
    nb = L.smc2_pf_workspace_bytes(ctypes.byref(cfg), runs)
    if c["runs"][0]["T"] >= 1:
        assert nb >= 256, c
    else:
        assert nb == 0 and L.smc2_last_error(None), c
    nb = L.smc2_pmcmc_workspace_bytes(ctypes.byref(cfg), 64, 100, runs)
    if nb == 0:
        assert L.smc2_last_error(None), c
    else:
        assert _valid_common(dict(c, runs=c["runs"][:1])), c
