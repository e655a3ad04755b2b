"""The truncated Langevin proposal on the GPU sampler (SMC2_PROP_LANGEVIN), through the C
ABI: the filters' score launches feed each sample's score estimate to the next
iteration's drift, and the proposal's exact log q enters the weights.

* Free-running parity with the reference sampler on the same streams: every iteration's
  proposals, log-likelihoods, pre-resampling log-weights, ancestors and records, the
  proposals' scores. The proposal covariance is the Cholesky factor of the proposing
  population's weighted covariance, summed in a different order on each side; the factor
  of a poorly conditioned covariance (few distinct samples after a resampling, a logit
  coordinate with a tiny spread) amplifies that rounding, so the proposals agree to 1e-9
  rather than the random walk's 1e-12; ancestors are identical.
* The scores travel with their samples: after a step the population's scores are the
  proposals' scores gathered by the ancestors.
* The GPU sampler with it reaches the exact grid posterior of the tiny SIR problem.
"""
import numpy as np
import pytest

import oracle as O
import paper_2311_12973_amd as G
from paper_2311_12973_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _run_pair(w, N, K, nx, T=None, seed=1, lkernel=None, prec=None, step=0.0):
    w = dict(w, proposal=G.PROP_LANGEVIN, lgv_step=step)
    if T is not None:
        w["T"] = T
    if lkernel is not None:
        w["lkernel"] = lkernel
    if prec is not None:
        w["prec"] = prec
    y = W.observations(w)
    s = G.Sampler(w, [dict(T=y.shape[0], nx=nx, seed=seed, y=y)], N=N, K=K)
    gpu = dict(phi=[], ll=[], lp=[], logw=[], anc=[], score_new=[], score=[], logq=[], theta=[])
    for k in range(K):
        s.step()
        for key, what in (("phi", "phi_new"), ("ll", "ll_new"), ("lp", "lp_new"), ("logw", "logw_pre"),
                          ("anc", "anc"), ("score_new", "score_new"), ("score", "score"), ("logq", "logq"),
                          ("theta", "theta_new")):
            gpu[key].append(s.dump(what))
    gpu = {k: np.array(v) for k, v in gpu.items()}
    gpu["rec"] = s.records()
    gpu["est"] = s.estimate(recycled=True)
    s.close()
    cfg = O.config_from_workload(w)
    ref = O.smc2_run(cfg, y, nx, seed, N, K, dumps=True)
    return gpu, ref, cfg, y


def _compare(gpu, ref, D, tol_ll):
    assert ref["status"] == 0
    K = gpu["ll"].shape[0]
    worst = dict(phi=0.0, ll=0.0, logw=0.0)
    for k in range(K):
        dphi = np.abs(gpu["phi"][k] - ref["phi"][k]) / np.maximum(1.0, np.abs(ref["phi"][k]))
        worst["phi"] = max(worst["phi"], float(dphi.max()))
        assert dphi.max() <= 1e-9, k
        assert np.allclose(gpu["lp"][k], ref["lp"][k], rtol=1e-9, atol=1e-9), k
        fin = np.isfinite(ref["ll"][k])
        assert np.array_equal(np.isfinite(gpu["ll"][k]), fin), k
        rel = np.abs(gpu["ll"][k][fin] - ref["ll"][k][fin]) / np.abs(ref["ll"][k][fin])
        worst["ll"] = max(worst["ll"], float(rel.max()) if rel.size else 0.0)
        assert rel.max() <= tol_ll, k
        fin = np.isfinite(ref["logw"][k])
        assert np.array_equal(np.isfinite(gpu["logw"][k]), fin), k
        dl = np.abs(gpu["logw"][k][fin] - ref["logw"][k][fin]) / np.maximum(1.0, np.abs(ref["logw"][k][fin]))
        worst["logw"] = max(worst["logw"], float(dl.max()))
        assert dl.max() <= 1e-7, k
        assert np.array_equal(gpu["anc"][k], ref["anc"][k]), k
    for col in [0, 2, 3, 4]:
        assert np.array_equal(gpu["rec"][:, col], ref["rec"][:, col]), col
    assert np.allclose(gpu["rec"][:, 1], ref["rec"][:, 1], rtol=1e-7)
    assert np.allclose(gpu["rec"][:, 6:], ref["rec"][:, 6:], rtol=1e-7, atol=1e-12)
    m_ref, _, _ = O.recycle(ref["rec"], D)
    assert np.allclose(gpu["est"][0], m_ref, rtol=1e-7)
    _log("  largest differences: proposals %.3g, estimates %.3g, log-weights %.3g" % (worst["phi"], worst["ll"],
                                                                                     worst["logw"]))


@pytest.mark.parametrize("name,N,K,nx,T,lkernel,prec,tol_ll,step", [
    ("sir_fp64", 64, 5, 64, None, None, None, 1e-9, 0.0),
    ("seir", 256, 4, 128, 40, G.L_FORWARD, None, 1e-4, 0.0),
    ("seir_learned", 128, 4, 96, 30, None, G.PREC_FP64, 1e-9, 0.0),
    ("seir_learned", 128, 4, 96, 30, None, G.PREC_FP64, 1e-9, 1.0),
])
def test_langevin_sampler_matches_reference(name, N, K, nx, T, lkernel, prec, tol_ll, step):
    w = W.preset(name)
    _log("Langevin %s N=%d K=%d nx=%d step=%g" % (name, N, K, nx, step))
    gpu, ref, cfg, y = _run_pair(w, N, K, nx, T=T, lkernel=lkernel, prec=prec, step=step)
    _compare(gpu, ref, w["D"], tol_ll)
    assert np.all(gpu["rec"][1:, -2] == 2) and gpu["rec"][0, -2] == 0
    # the proposals' scores: the reference's score estimates of the same filters
    for k in range(K):
        fin = np.isfinite(gpu["ll"][k])
        for i in np.flatnonzero(fin)[:8]:
            sc = O.pf_score(cfg, gpu["theta"][k][i], y, nx, 1, int(i), k + 1)[1]
            scale = np.maximum(1.0, np.abs(sc))
            assert np.all(np.abs(gpu["score_new"][k][i] - sc) <= 1e-9 * scale), (k, i)
        # scores travel with their samples through resampling
        assert np.array_equal(gpu["score"][k], gpu["score_new"][k][gpu["anc"][k]])


def test_gpu_langevin_sampler_targets_the_grid_posterior():
    from tests.test_oracle_mlp import I0, MED, N_POP, SD, _grid_posterior
    y, grid_mean, grid_sd = _grid_posterior()
    prior = [[W.PRIOR_LOGNORMAL, np.log(MED[0]), SD], [W.PRIOR_LOGNORMAL, np.log(MED[1]), SD]]
    w = dict(model=W.SIR, obs=W.OBS_POIS_PREV, D=2, prec=W.PREC_FP64, n_pop=N_POP, fixed=[I0], prior=prior,
             rw_cov=(0.05 * np.eye(2)).tolist(), lkernel=G.L_FORWARD, proposal=G.PROP_LANGEVIN)
    R = 24
    runs = [dict(T=y.shape[0], nx=48, seed=s, y=y) for s in range(1, R + 1)]
    smp = G.Sampler(w, runs, N=1024, K=8)
    for _ in range(8):
        smp.step()
    ests = np.array([smp.estimate(r)[0] for r in range(R)])
    second = np.array([np.diag(smp.estimate(r)[1]) + smp.estimate(r)[0] ** 2 for r in range(R)])
    smp.close()
    se = ests.std(0, ddof=1) / np.sqrt(R)
    pooled_sd = np.sqrt(second.mean(0) - ests.mean(0) ** 2)
    _log("GPU Langevin: posterior mean %s (grid %s, s.e. %s), sd %s (grid %s)"
         % (ests.mean(0), grid_mean, se, pooled_sd, grid_sd))
    assert np.all(np.abs(ests.mean(0) - grid_mean) < 4 * se + 2e-3)
    assert np.all(np.abs(pooled_sd / grid_sd - 1) < 0.2)


@pytest.mark.parametrize("schedule", [G.SCHED_AUTO, G.SCHED_POOLED])
def test_langevin_score_launches_identical_under_every_launch(schedule):
    """Score launches with several filters per workgroup: a persistent grid (automatic for
    2048 filters of 1024 particles, four rounds of resident workgroups) and a workgroup per
    filter give the same records, likelihoods and scores, under either draw schedule. (The
    score's chunk sums once started without waiting for every wave to finish reading the
    last day's weight sums from the same slots; a lagging wave could then take a wrong sum,
    which showed as a diverging run under the persistent grid.)"""
    w = dict(W.preset("seir_learned"), T=30, proposal=G.PROP_LANGEVIN)
    y = W.observations(w)
    run = [dict(T=30, nx=1024, seed=7, y=y)]
    out = {}
    for launch in (G.LAUNCH_PER_FILTER, G.LAUNCH_AUTO, G.LAUNCH_PERSISTENT):
        s = G.Sampler(w, run, N=2048, K=4, persistent=launch, schedule=schedule)
        dumps = []
        for _ in range(4):
            s.step()
            dumps.append((s.dump("ll_new"), s.dump("score_new"), s.dump("anc"), s.dump("phi_new")))
        out[launch] = (s.records(), dumps, s.groups())
        s.close()
    _log("schedule %d groups: per filter %s, automatic %s" % (schedule, out[G.LAUNCH_PER_FILTER][2],
                                                               out[G.LAUNCH_AUTO][2]))
    assert all(g["persistent"] == 1 for g in out[G.LAUNCH_AUTO][2])
    ref = out[G.LAUNCH_PER_FILTER]
    for launch in (G.LAUNCH_AUTO, G.LAUNCH_PERSISTENT):
        got = out[launch]
        assert np.array_equal(got[0], ref[0]), launch
        for a, b in zip(got[1], ref[1]):
            for x, z in zip(a, b):
                assert np.array_equal(np.nan_to_num(x, neginf=-1e300), np.nan_to_num(z, neginf=-1e300)), launch
