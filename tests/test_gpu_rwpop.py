"""The random walk with the population's covariance on the GPU sampler
(SMC2_PROP_RW_POP), through the C ABI. Its proposal covariance is the Cholesky factor of
the proposing population's weighted covariance (one workgroup per run before the
proposals); it needs no score, so the filters keep their configured schedule (the
pooled one included) and every model runs it.

* Free-running parity with the reference sampler on the same streams: every iteration's
  proposals, log-likelihoods, pre-resampling log-weights, ancestors, records and the
  recycled estimate. The two sides sum the covariance in different orders and its factor
  amplifies that rounding for a poorly conditioned population, so proposals agree to
  1e-9; ancestors are identical.
* The proposals' log q dumped by the GPU equals log N(phi_new; phi, Sigma_pop), Sigma_pop
  the weighted covariance of the dumped population (numpy, with the degenerate
  population's diagonal fallback).
* The GPU sampler with it reaches the exact grid posterior of the tiny SIR problem.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
import paper_2311_12973_amd as G
from paper_2311_12973_amd import workloads as W
from tests.test_gpu_langevin import _compare
from tests.test_oracle_rwpop import _factor

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _run_pair(w, N, K, nx, sched, seed=1):
    y = W.observations(w)
    s = G.Sampler(w, [dict(T=y.shape[0], nx=nx, seed=seed, y=y)], N=N, K=K, schedule=sched)
    gpu = dict(phi=[], ll=[], lp=[], logw=[], anc=[], logq=[], pop=[], pop_logw=[])
    for k in range(K):
        gpu["pop"].append(s.dump("phi"))
        gpu["pop_logw"].append(s.dump("logw"))
        s.step()
        for key, what in (("phi", "phi_new"), ("ll", "ll_new"), ("lp", "lp_new"), ("logw", "logw_pre"),
                          ("anc", "anc"), ("logq", "logq")):
            gpu[key].append(s.dump(what))
    gpu = {k: np.array(v) for k, v in gpu.items()}
    gpu["rec"] = s.records()
    gpu["est"] = s.estimate(recycled=True)
    s.close()
    cfg = O.config_from_workload(w)
    ref = O.smc2_run(cfg, y, nx, seed, N, K, dumps=True)
    return gpu, ref


CASES = [  # workload, overrides, N, K, nx, filter schedule
    ("sir_fp64", dict(T=30), 64, 5, 64, G.SCHED_AUTO),
    ("seir", dict(T=40, lkernel=G.L_FORWARD), 256, 4, 128, G.SCHED_AUTO),
    ("seir", dict(T=40), 256, 4, 96, G.SCHED_POOLED),
    ("seir_learned", dict(T=30, prec=G.PREC_FP64), 128, 4, 96, G.SCHED_PER_DRAW),
    ("age_seir", dict(T=12), 48, 3, 64, G.SCHED_AUTO),
    ("sir_fp64", dict(T=30, pf_resampling=G.PF_RS_MULTINOMIAL, pf_always=1), 64, 4, 64, G.SCHED_AUTO),
]


@pytest.mark.parametrize("name,over,N,K,nx,sched", CASES)
def test_population_walk_matches_reference(name, over, N, K, nx, sched):
    w = dict(W.preset(name), proposal=G.PROP_RW_POP, **over)
    _log("population random walk %s %s N=%d K=%d nx=%d schedule=%d" % (name, over, N, K, nx, sched))
    gpu, ref = _run_pair(w, N, K, nx, sched)
    tol_ll = 1e-9 if w["prec"] == G.PREC_FP64 else 1e-4
    _compare(gpu, ref, w["D"], tol_ll)
    assert np.all(gpu["rec"][1:, -2] == 3) and gpu["rec"][0, -2] == 0
    # log q of each proposal from its definition, at the population it was proposed from
    for k in range(1, K):
        pop, lw = gpu["pop"][k], gpu["pop_logw"][k]
        fin = np.isfinite(lw)
        wn = np.where(fin, np.exp(lw - lw[fin].max()), 0.0)
        wn /= wn.sum()
        mu = wn @ pop
        L = _factor((pop - mu).T @ ((pop - mu) * wn[:, None]), mu)
        for i in range(0, N, max(1, N // 16)):
            want = stats.multivariate_normal(pop[i], L @ L.T).logpdf(gpu["phi"][k][i])
            assert gpu["logq"][k][i] == pytest.approx(want, rel=1e-8, abs=1e-8), (k, i)


def test_gpu_population_walk_targets_the_grid_posterior():
    from tests.test_oracle_mlp import I0, MED, N_POP, SD, _grid_posterior
    y, grid_mean, grid_sd = _grid_posterior()
    prior = [[W.PRIOR_LOGNORMAL, np.log(MED[0]), SD], [W.PRIOR_LOGNORMAL, np.log(MED[1]), SD]]
    w = dict(model=W.SIR, obs=W.OBS_POIS_PREV, D=2, prec=W.PREC_FP64, n_pop=N_POP, fixed=[I0], prior=prior,
             rw_cov=(0.05 * np.eye(2)).tolist(), lkernel=G.L_GAUSS_OPT, proposal=G.PROP_RW_POP)
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
    _log("GPU population random walk: posterior mean %s (grid %s, s.e. %s), sd %s (grid %s)"
         % (ests.mean(0), grid_mean, se, pooled_sd, grid_sd))
    assert np.all(np.abs(ests.mean(0) - grid_mean) < 4 * se + 2e-3)
    assert np.all(np.abs(pooled_sd / grid_sd - 1) < 0.2)


@pytest.mark.parametrize("proposal", [G.PROP_RW_POP, G.PROP_LANGEVIN])
def test_population_covariance_batched_under_every_launch_configuration(proposal):
    """Uneven runs in one context with the population-covariance proposals: each run's
    covariance factor comes from its own population (one workgroup per run), and a
    persistent grid, the autotuned configuration and a replayed graph of the persistent
    grid give results identical to the default launch."""
    from tests.test_gpu_sampler import _batched_dumps
    w = dict(W.preset("seir_batched"), proposal=proposal)
    runs = W.batched_runs(w, n_runs=4)
    _log("proposal %d, runs: %s" % (proposal, ", ".join("T=%d nx=%d" % (r["T"], r["nx"]) for r in runs)))
    base, _ = _batched_dumps(w, runs, 32, 3)
    for over in (dict(persistent=1), dict(tune=1), dict(persistent=1, use_graph=1)):
        other, _ = _batched_dumps(w, runs, 32, 3, **over)
        for key in ("ll", "logw", "anc", "rec"):
            assert np.array_equal(np.nan_to_num(base[key], neginf=-1e300),
                                  np.nan_to_num(other[key], neginf=-1e300)), (over, key)
    assert np.all(base["rec"][:, 1:, -2] == (3 if proposal == G.PROP_RW_POP else 2))


def test_population_walk_batched_matches_reference_per_run():
    """Three uneven runs of the batched workload in one context against the reference
    sampler run by run: the records of every iteration."""
    w = dict(W.preset("seir_batched"), proposal=G.PROP_RW_POP)
    runs = W.batched_runs(w, n_runs=3)
    K = 3
    s = G.Sampler(w, runs, N=32, K=K)
    for _ in range(K):
        s.step()
    recs = [s.records(r) for r in range(len(runs))]
    s.close()
    cfg = O.config_from_workload(w)
    for r, run in enumerate(runs):
        _log("run %d: T=%d nx=%d" % (r, run["T"], run["nx"]))
        ref = O.smc2_run(cfg, run["y"], run["nx"], run["seed"], 32, K)
        assert ref["status"] == 0
        assert np.array_equal(recs[r][:, [0, 2, 3, 4, -2]], ref["rec"][:, [0, 2, 3, 4, -2]])
        assert np.allclose(recs[r][:, 6:], ref["rec"][:, 6:], rtol=1e-4, atol=1e-10)


@pytest.mark.parametrize("N", [2, 32768])
def test_population_walk_sample_count_limits(N):
    """The smallest and largest sample counts the interface accepts, against the reference
    sampler: with two samples the population's covariance is singular after every
    resampling (the diagonal fallback), with 32768 one workgroup per run sums it over the
    whole population."""
    w = dict(W.preset("seir"), T=10, proposal=G.PROP_RW_POP, prec=G.PREC_FP64)
    _log("population random walk N=%d" % N)
    gpu, ref = _run_pair(w, N, 3, 16, G.SCHED_AUTO)
    _compare(gpu, ref, w["D"], 1e-9)
    assert np.all(gpu["rec"][1:, -2] == 3)
