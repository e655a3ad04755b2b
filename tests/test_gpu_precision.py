"""Precision of the GPU path against the FP64 reference, and the executed-work counter.

* FP32 filters (per-step weights in FP32, cross-time accumulation in FP64) against the
  FP64 reference on the same random streams:
  - free running, each side taking its own integer decisions: the relative error of
    the log-likelihood and the fraction of filters whose decisions (counts, resampling
    flags, ancestors) differ anywhere;
  - with the GPU's decisions injected into the FP64 reference (its replay of Sec. II's
    weights): the relative error of the log-likelihood must be <= 1e-4. Filters whose
    decisions agree reproduce the free-running FP64 estimate exactly in the replay.
* The FP64 outer step against the reference recomputing it from the GPU's inputs: the
  L-kernel fit's weighted moments and the log-weights.
* End to end: every filter of a sampler iteration replayed in FP64 on the GPU's
  decisions, and the reference's outer step on the replayed estimates: posterior means
  and ESS within 1e-4 of the GPU's.
* The executed particle-steps of a run (N_x x days each active filter ran, stopping at
  a filter's death day) against the reference's filters.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle as O
import paper_2311_12973_amd as G
from paper_2311_12973_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def fp32_precision(w, theta, y, nx, seed, k, threads=16):
    """GPU FP32 filters against the FP64 reference on the same streams (free running and
    replaying the GPU's decisions). Returns a dict of per-filter arrays."""
    ll32, _, rs, st, anc = G.pf_trace_state(w, theta, y, nx, seed, k, precision=G.PREC_FP32, with_anc=True)
    cfg64 = O.config_from_workload(w, prec=O.PREC_FP64)

    def one(i):
        ll64, _, rs64, st64, anc64 = O.pf_trace_full(cfg64, theta[i], y, nx, seed, i, k)
        rep, _ = O.pf_replay(cfg64, theta[i], y, st[i], anc[i], rs[i])
        # first day whose decisions differ (counts, resampling flag, ancestors); T when none
        days = len(y) if np.isfinite(ll32[i]) and np.isfinite(ll64) else 0
        first = days
        for t in range(days):
            if (rs64[t] != rs[i][t] or not np.array_equal(st64[t], st[i][t])
                    or (rs[i][t] and not np.array_equal(anc64[t], anc[i][t]))):
                first = t
                break
        same = np.isfinite(ll64) == np.isfinite(ll32[i]) and first == days and days > 0
        return ll64, rep, same, first

    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, range(len(theta))))
    ll64 = np.array([r[0] for r in res])
    rep = np.array([r[1] for r in res])
    same = np.array([r[2] for r in res])
    first = np.array([r[3] for r in res])
    return dict(ll32=ll32, ll64=ll64, replay=rep, same=same, first_divergence_day=first)


def _theta(w, n, seed, scale=0.1):
    rng = np.random.default_rng(seed)
    th = np.array(w["truth"]) * np.exp(rng.normal(0, scale, size=(n, w["D"])))
    th[:, 3] = np.clip(th[:, 3], 1e-7, 1e-3)
    return th


@pytest.mark.parametrize("name,nx,T,n", [("seir", 512, 100, 48), ("age_seir", 256, 120, 16)])
def test_fp32_filters_against_the_fp64_reference(name, nx, T, n):
    w = dict(W.preset(name), T=T)
    y = W.observations(w)
    theta = _theta(w, n, 3)
    r = fp32_precision(w, theta, y, nx, seed=17, k=4)
    fin = np.isfinite(r["ll64"]) & np.isfinite(r["ll32"])
    assert fin.sum() >= n // 2
    free = np.abs(r["ll32"][fin] - r["ll64"][fin]) / np.abs(r["ll64"][fin])
    fin_r = np.isfinite(r["replay"])
    assert np.array_equal(fin_r, np.isfinite(r["ll32"]))
    rep = np.abs(r["ll32"][fin_r] - r["replay"][fin_r]) / np.abs(r["replay"][fin_r])
    _log("%s: free-running rel err median %.3g max %.3g; decisions differ in %d/%d filters (first at day %s of "
         "%d, median); replayed rel err median %.3g max %.3g" % (
             name, np.median(free), free.max(), (~r["same"]).sum(), n, np.median(r["first_divergence_day"]) + 1,
             T, np.median(rep), rep.max()))
    assert rep.max() <= 1e-4
    agree = r["same"] & fin
    assert np.array_equal(r["replay"][agree], r["ll64"][agree])


@pytest.mark.parametrize("proposal", [G.PROP_RW, G.PROP_MLP])
def test_outer_step_fp64_against_the_reference(proposal):
    w = dict(W.preset("seir_learned"), T=40, proposal=proposal, mlp_epochs=2, mlp_batch=256, mlp_lr=3e-3)
    y = W.observations(w)
    N, K, nx = 1024, 4, 128
    s = G.Sampler(w, [dict(T=y.shape[0], nx=nx, seed=5, y=y)], N=N, K=K)
    cfg = O.config_from_workload(w)
    errs = dict(mu=0.0, cov=0.0, logw=0.0)
    for k in range(1, K + 1):
        before = {key: s.dump(key) for key in ("phi", "lp", "ll", "logw")}
        s.step()
        if k == 1:
            continue
        rec = s.records()[k - 1]
        phin, lpn, lln, lwp = (s.dump(x) for x in ("phi_new", "lp_new", "ll_new", "logw_pre"))
        lq = s.dump("logq") if rec[G.record_len(w["D"]) - 2] else None
        om = np.exp(before["logw"] - np.max(before["logw"]))
        om /= om.sum()
        _, mu, cov = O.lkernel_fit_cov(before["phi"], phin, om)
        fit = s.dump("lkfit")
        D2 = 2 * w["D"]
        errs["mu"] = max(errs["mu"], np.max(np.abs(fit[:D2] - mu) / np.maximum(np.abs(mu), 1e-300)))
        errs["cov"] = max(errs["cov"], np.max(np.abs(fit[D2:].reshape(D2, D2) - cov)) / np.max(np.abs(cov)))
        st, lwp_ref, anc_ref, _ = O.outer_update(cfg, k, 5, dict(before), phin, lpn, lln, lq)
        fin = np.isfinite(lwp_ref)
        assert np.array_equal(np.isfinite(lwp), fin)
        errs["logw"] = max(errs["logw"], np.max(np.abs(lwp[fin] - lwp_ref[fin]) / np.maximum(np.abs(lwp_ref[fin]), 1)))
        assert np.array_equal(s.dump("anc"), anc_ref)
    s.close()
    _log("outer step (proposal %d): L-kernel mean rel err %.3g, covariance %.3g (of its largest entry), "
         "log-weights %.3g" % (proposal, errs["mu"], errs["cov"], errs["logw"]))
    assert errs["mu"] <= 1e-12 and errs["cov"] <= 1e-12 and errs["logw"] <= 1e-9


def test_end_to_end_replay_posterior_means():
    """The end-to-end level of the replay: every filter of each iteration (FP32 on the
    GPU) is traced on the same streams through the kernel-level entry point (which
    reproduces the sampler's estimate bit for bit), its weights are recomputed in FP64 by
    the reference on the GPU's decisions, and the reference's outer step on those
    estimates gives the iteration's posterior mean and ESS: within 1e-4 of the GPU's."""
    w = dict(W.preset("seir"), T=40)
    y = W.observations(w)
    N, K, nx, seed = 256, 3, 256, 5
    s = G.Sampler(w, [dict(T=y.shape[0], nx=nx, seed=seed, y=y)], N=N, K=K)
    cfg = O.config_from_workload(w)
    cfg64 = O.config_from_workload(w, prec=O.PREC_FP64)
    D = w["D"]
    worst = dict(ll=0.0, mean=0.0, ess=0.0)
    for k in range(1, K + 1):
        before = {key: s.dump(key) for key in ("phi", "lp", "ll", "logw")}
        s.step()
        rec = s.records()[k - 1]
        theta, phin, lpn, lln = (s.dump(x) for x in ("theta_new", "phi_new", "lp_new", "ll_new"))
        ll32, _, rs, st, anc = G.pf_trace_state(w, theta, y, nx, seed, k, precision=G.PREC_FP32, with_anc=True)
        act = np.isfinite(lln)
        assert np.array_equal(ll32[act], lln[act])

        def replay(i):
            return O.pf_replay(cfg64, theta[i], y, st[i], anc[i], rs[i])[0] if act[i] else -np.inf

        with cf.ThreadPoolExecutor(8) as ex:
            ll_rep = np.array(list(ex.map(replay, range(N))))
        fin = np.isfinite(ll_rep)
        assert np.array_equal(fin, act)
        worst["ll"] = max(worst["ll"], float(np.max(np.abs(lln[fin] - ll_rep[fin]) / np.abs(ll_rep[fin]))))
        st_ref = dict(phi=np.zeros((N, D)), lp=np.zeros(N), ll=np.zeros(N), logw=np.zeros(N)) if k == 1 else before
        status, _, _, rec_ref = O.outer_update(cfg, k, seed, dict(st_ref), phin, lpn, ll_rep)
        assert status == 0
        worst["mean"] = max(worst["mean"], float(np.max(np.abs(rec[6:6 + D] - rec_ref[6:6 + D])
                                                       / np.abs(rec_ref[6:6 + D]))))
        worst["ess"] = max(worst["ess"], abs(rec[1] - rec_ref[1]) / rec_ref[1])
    s.close()
    _log("end-to-end replay: log-likelihoods %.3g, posterior means %.3g, ESS %.3g (largest relative differences)"
         % (worst["ll"], worst["mean"], worst["ess"]))
    assert worst["ll"] <= 1e-4 and worst["mean"] <= 1e-4 and worst["ess"] <= 1e-4


def test_executed_particle_steps_counter():
    """Small filters (N_x = 4) with Poisson observations of new cases: some filters lose
    every particle before the last day and stop there."""
    w = W.preset("sir_fp64")
    y = W.observations(w)
    N, K, nx, T = 64, 3, 4, y.shape[0]
    s = G.Sampler(w, [dict(T=T, nx=nx, seed=1, y=y)], N=N, K=K)
    cfg = O.config_from_workload(w)
    want, died = 0, 0
    for k in range(1, K + 1):
        logw_prev = s.dump("logw")
        s.step()
        lpn, lln = s.dump("lp_new"), s.dump("ll_new")
        theta = np.array([O.theta_of_phi(cfg, p) for p in s.dump("phi_new")])
        for i in range(N):
            if not (k == 1 or (logw_prev[i] != -np.inf and lpn[i] != -np.inf)):
                continue
            days = T
            if lln[i] == -np.inf:
                _, inc, _ = O.pf_loglik(cfg, theta[i], y, nx, 1, i, k, trace=True)
                days = int(np.flatnonzero(inc == -np.inf)[0]) + 1
                died += days < T
            want += nx * days
    got = int(s.dump("psteps")[0])
    s.close()
    _log("executed particle-steps %d (nominal %d), filters stopped early %d" % (got, K * N * nx * T, died))
    assert died > 0
    assert got == want
