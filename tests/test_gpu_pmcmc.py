"""GPU particle marginal Metropolis-Hastings (Sec. III, Eq. MHalgorithm_) against the
reference, through the C ABI.

* FP64 filters: the chains' states, likelihood estimates and decisions equal the
  reference's run on the same streams (states and estimates to 1e-12 / 1e-10).
* FP32 filters: every decision replayed by the reference from the GPU's trace: the
  random-walk proposal recomputed from the previous state (equal to the next state where
  accepted), the proposal's filter estimate against the reference FP32 filter (1e-4), and
  the Metropolis-Hastings decision from the GPU's estimates and the stream's uniform.
* The GPU chains target the exact grid posterior of the tiny SIR problem (four-particle
  estimates), like the reference's pin.
"""
import numpy as np
import pytest

import oracle as O
import paper_2311_12973_amd as G
from paper_2311_12973_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def test_pmcmc_fp64_matches_reference():
    w = W.preset("sir_fp64")
    y = W.observations(w)
    C, I, nx, seed = 24, 40, 64, 5
    mc = G.PMCMC(w, dict(T=y.shape[0], nx=nx, seed=seed, y=y), C, I)
    mc.step(15)
    mc.step(I - 15)
    phi, ll, acc = mc.dump("phi"), mc.dump("ll"), mc.dump("accepted")
    mean, cov, rate = mc.estimate(I // 2)
    mc.close()
    cfg = O.config_from_workload(w)
    th_ref, ll_ref, acc_ref = O.pmcmc_run(cfg, y, nx, seed, C, I)
    th = np.array([[O.theta_of_phi(cfg, p) for p in chain] for chain in phi])
    _log("acceptance %.3f (reference %.3f)" % (acc.mean(), acc_ref.mean()))
    assert np.array_equal(acc, acc_ref)
    assert np.allclose(th, th_ref, rtol=1e-12, atol=0)
    fin = np.isfinite(ll_ref)
    assert np.array_equal(np.isfinite(ll), fin)
    assert np.allclose(ll[fin], ll_ref[fin], rtol=1e-10)
    post = th_ref[:, 1 + I // 2:, :].reshape(-1, w["D"])
    assert np.allclose(mean, post.mean(0), rtol=1e-10)
    assert np.allclose(cov, np.cov(post.T, bias=True), rtol=1e-8, atol=1e-14)
    assert rate == pytest.approx(acc_ref[:, I // 2:].mean(), rel=1e-12)


def test_pmcmc_fp32_decisions_replayed_by_reference():
    w = dict(W.preset("seir"), T=60)
    y = W.observations(w)
    C, I, nx, seed = 16, 20, 256, 7
    mc = G.PMCMC(w, dict(T=y.shape[0], nx=nx, seed=seed, y=y), C, I)
    mc.step(I)
    phi, ll, lln, acc = mc.dump("phi"), mc.dump("ll"), mc.dump("ll_proposed"), mc.dump("accepted")
    mc.close()
    cfg = O.config_from_workload(w, prec=O.PREC_FP32)
    st, L = O.cholesky(np.asarray(w["rw_cov"]))
    assert st == 0
    worst = 0.0
    for c in range(C):
        for m in range(1, I + 1):
            z = np.array([O.normal_call(seed, [c, 0, m << 16, (9 << 24) | d]) for d in range(w["D"])])
            phn = phi[c, m - 1] + L @ z
            lp, lpn = O.prior_logpdf(cfg, phi[c, m - 1]), O.prior_logpdf(cfg, phn)
            if lpn == -np.inf:
                assert lln[c, m - 1] == -np.inf
            else:
                ref = O.pf_loglik(cfg, O.theta_of_phi(cfg, phn), y, nx, seed, c, m)
                if np.isfinite(ref):
                    worst = max(worst, abs(lln[c, m - 1] - ref) / abs(ref))
                else:
                    assert lln[c, m - 1] == -np.inf
            wd = O.philox([c, 0, m << 16, 10 << 24], [seed & 0xFFFFFFFF, seed >> 32])
            u = O.u53(wd[0], wd[1])
            assert O.mh_accept(lp, ll[c, m - 1], lpn, lln[c, m - 1], u) == bool(acc[c, m - 1]), (c, m)
            if acc[c, m - 1]:
                assert np.allclose(phi[c, m], phn, rtol=1e-13, atol=1e-15)
                assert ll[c, m] == lln[c, m - 1]
            else:
                assert np.array_equal(phi[c, m], phi[c, m - 1]) and ll[c, m] == ll[c, m - 1]
    _log("FP32 p-MCMC: acceptance %.3f, proposals' estimates within %.3g of the reference" % (acc.mean(), worst))
    assert worst <= 1e-4


def test_pmcmc_targets_the_grid_posterior():
    from tests.test_oracle_mlp import MED, SD, _grid_posterior
    y, gm, gsd = _grid_posterior()
    prior = [[W.PRIOR_LOGNORMAL, np.log(MED[0]), SD], [W.PRIOR_LOGNORMAL, np.log(MED[1]), SD]]
    w = dict(model=W.SIR, obs=W.OBS_POIS_PREV, D=2, prec=W.PREC_FP64, n_pop=12, fixed=[2], prior=prior,
             rw_cov=(0.1 * np.eye(2)).tolist())
    C, I, burn = 256, 600, 150
    mc = G.PMCMC(w, dict(T=y.shape[0], nx=4, seed=11, y=y), C, I)
    mc.step(I)
    phi = mc.dump("phi")
    mean, cov, rate = mc.estimate(burn)
    mc.close()
    th = np.exp(phi[:, 1 + burn:, :])
    cm = th.mean(1)
    se = cm.std(0, ddof=1) / np.sqrt(C)
    _log("GPU p-MCMC posterior mean %s (grid %s, s.e. %s), sd %s (grid %s), acceptance %.3f"
         % (cm.mean(0), gm, se, np.sqrt(np.diag(cov)), gsd, rate))
    assert np.allclose(mean, th.reshape(-1, 2).mean(0), rtol=1e-12)
    assert np.all(np.abs(cm.mean(0) - gm) < 4 * se + 2e-3)
    assert np.all(np.abs(np.sqrt(np.diag(cov)) / gsd - 1) < 0.1)
