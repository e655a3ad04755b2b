"""The scalar linear-Gaussian model on the GPU particle-filter kernel (FP64), through
the C ABI. Its likelihood has a closed form (the Kalman filter), so the kernel's
model-independent steps of Sec. II (weight recursion, likelihood increments with the
mean-weight reset, the exact ESS trigger, systematic and multinomial ancestors) are
pinned on the GPU itself, besides the parity with the reference:

* parity: likelihood estimates, per-day increments, resampling flags and states equal
  the reference filter's on the same streams (flags exactly, the rest to FP64 rounding
  of the transcendentals), over ragged particle counts, several iterations' streams,
  both resampling schemes and resampling at every step;
* the deterministic special case (no state noise): the exact likelihood and the
  states a^t m0, bit for bit;
* unbiasedness: the mean of exp(ll - ll_Kalman) over thousands of GPU filters is 1;
* the whole GPU sampler (outer step, L-kernel, recycling) on this model reaches the
  exact posterior computed from the Kalman likelihood on a grid, with the random walk,
  the learned proposal, the population random walk and the Langevin proposal (its
  score launches on this model).
"""
import numpy as np
import pytest

import oracle as O
import paper_2311_12973_amd as G
from paper_2311_12973_amd import workloads as W
from tests.exact_models import kalman_loglik_grid

pytestmark = pytest.mark.gpu

# |a| < 1 in every row: the device's and the host library's FP64 log and cos in the
# Box-Muller draws may differ in the last bit, and a state carries its rounding forward
# multiplied by a each day (by 1.02^1000 = 4e8 over the longest case for a = 1.02)
THETAS = np.array([[0.9, 1.0, 1.0], [0.5, 0.3, 2.0], [-0.7, 1.5, 0.4], [0.99, 0.8, 1.1], [0.0, 2.0, 0.25]])


def _log(msg):
    print(msg, flush=True)


def _states(st):
    """int32 [n][T][2][nx] (low, high words) -> float64 [n][T][nx]"""
    lo = st[:, :, 0, :].astype(np.uint32).astype(np.uint64)
    hi = st[:, :, 1, :].astype(np.uint32).astype(np.uint64)
    return ((hi << np.uint64(32)) | lo).view(np.float64)


CASES = [  # T, nx, k, resampling, pf_always, block
    (25, 64, 0, G.PF_RS_SYSTEMATIC, 0, 0),
    (100, 1000, 3, G.PF_RS_SYSTEMATIC, 0, 256),
    (40, 257, 2, G.PF_RS_MULTINOMIAL, 0, 0),
    (30, 100, 1, G.PF_RS_SYSTEMATIC, 1, 64),
    (1, 1, 0, G.PF_RS_SYSTEMATIC, 0, 0),
    (12, 4096, 5, G.PF_RS_SYSTEMATIC, 0, 0),
    (1024, 96, 7, G.PF_RS_MULTINOMIAL, 0, 0),
]


@pytest.mark.parametrize("T,nx,k,rs,always,block", CASES)
def test_filter_matches_reference(T, nx, k, rs, always, block):
    w = dict(W.preset("lingauss"), pf_resampling=rs, pf_always=always)
    y = W.simulate(W.LINGAUSS, W.OBS_GAUSS, 1.0, [0.9, 1.0, 1.0], T, 21 + T, w["fixed"])
    seed = 17
    _log("linear-Gaussian parity T=%d nx=%d k=%d resampling=%d always=%d block=%d" % (T, nx, k, rs, always, block))
    ll, inc, rsf, st = G.pf_trace_state(w, THETAS, y, nx, seed, k, block=block)
    xs = _states(st)
    m0, s0 = w["fixed"]
    for i, th in enumerate(THETAS):
        r_ll, r_inc, r_rs, r_x = O.pf_lg(th[0], th[1], th[2], m0, s0, y, nx, seed, filt=i, pf_always=always,
                                         trace=True, resampling=rs, k=k, states=True)
        di = np.abs(inc[i] - r_inc)
        dx = np.abs(xs[i] - r_x) / np.maximum(np.abs(r_x), 1e-300)
        bad = np.nonzero(di > 1e-9 + 1e-10 * np.abs(r_inc))[0]
        if bad.size:
            t0 = bad[0]
            _log("  filter %d: increments differ from day %d (%.3g vs %.3g); states' largest relative "
                 "difference before it %.3g, on it %.3g; resampling flags equal %s"
                 % (i, t0 + 1, inc[i, t0], r_inc[t0], dx[:t0].max() if t0 else 0.0, dx[t0].max(),
                    np.array_equal(rsf[i], r_rs)))
        assert np.array_equal(rsf[i], r_rs), i
        assert ll[i] == pytest.approx(r_ll, rel=1e-11, abs=1e-9), i
        assert not bad.size, i
        assert np.allclose(xs[i], r_x, rtol=1e-12, atol=1e-12), i
    _log("  resampling days %d of %d (filter 2)" % (rsf[2].sum(), T))


def test_deterministic_case_is_exact():
    w = W.preset("lingauss", fixed=[2.5, 0.0])
    y = W.simulate(W.LINGAUSS, W.OBS_GAUSS, 1.0, [0.8, 0.5, 0.7], 12, 5, [2.5, 0.0])
    th = np.array([[0.8, 0.0, 0.7], [-0.9, 0.0, 1.3]])
    ll, inc, rs, st = G.pf_trace_state(w, th, y, 96, 9, 3)
    xs = _states(st)
    for i in range(2):
        x, ref = 2.5, 0.0
        for t in range(len(y)):
            x = th[i, 0] * x
            assert np.all(xs[i, t] == x), (i, t)
            ref += -0.5 * np.log(2 * np.pi * th[i, 2] ** 2) - 0.5 * ((y[t] - x) / th[i, 2]) ** 2
        assert ll[i] == pytest.approx(ref, rel=1e-13)
    assert not rs.any()


@pytest.mark.parametrize("rs,always", [(G.PF_RS_SYSTEMATIC, 0), (G.PF_RS_MULTINOMIAL, 0), (G.PF_RS_SYSTEMATIC, 1)])
def test_gpu_estimate_is_unbiased_against_kalman(rs, always):
    w = dict(W.preset("lingauss"), pf_resampling=rs, pf_always=always)
    th = [0.9, 1.0, 1.0]
    y = W.simulate(W.LINGAUSS, W.OBS_GAUSS, 1.0, th, 25, 11, w["fixed"])
    ref = float(kalman_loglik_grid(th[0], th[1], th[2], w["fixed"][0], w["fixed"][1], y))
    M = 8000
    ll = G.pf_loglik(w, np.tile(th, (M, 1)), y, 64, 7, 2)
    r = np.exp(ll - ref)
    mean, se = r.mean(), r.std(ddof=1) / np.sqrt(M)
    _log("GPU linear-Gaussian filter: mean exp(ll - ll_Kalman) %.4f (s.e. %.4f), resampling %d always %d"
         % (mean, se, rs, always))
    assert abs(mean - 1.0) < 4 * se + 1e-3


def test_noalloc_entry_point_on_the_linear_gaussian_model():
    w = W.preset("lingauss")
    y = W.observations(w)
    a = G.pf_loglik(w, THETAS, y, 200, 3, 4)
    b = G.pf_loglik_noalloc(w, THETAS, y, 200, 3, 4)
    assert np.array_equal(a, b)


def grid_posterior(w, y, G_=48):
    """Exact posterior mean and standard deviation of theta: Kalman likelihood times the
    prior on a grid of the sampler coordinates, refined around a first coarse grid."""
    pr = np.array(w["prior"])
    m0, s0 = w["fixed"]

    def on(lo, hi, n):
        ax = [np.linspace(lo[d], hi[d], n) for d in range(3)]
        P = np.meshgrid(*ax, indexing="ij")
        th = [P[0], np.exp(P[1]), np.exp(P[2])]
        lw = kalman_loglik_grid(th[0], th[1], th[2], m0, s0, y)
        lw = lw + sum(-0.5 * ((P[d] - pr[d, 1]) / pr[d, 2]) ** 2 for d in range(3))
        wg = np.exp(lw - lw.max())
        wg /= wg.sum()
        mp = np.array([(wg * P[d]).sum() for d in range(3)])
        sp = np.sqrt([(wg * (P[d] - mp[d]) ** 2).sum() for d in range(3)])
        mt = np.array([(wg * th[d]).sum() for d in range(3)])
        stt = np.sqrt([(wg * (th[d] - mt[d]) ** 2).sum() for d in range(3)])
        return mp, sp, mt, stt

    mp, sp, _, _ = on(pr[:, 1] - 5 * pr[:, 2], pr[:, 1] + 5 * pr[:, 2], 40)
    _, _, mt, stt = on(mp - 7 * sp, mp + 7 * sp, G_)
    return mt, stt


@pytest.mark.parametrize("proposal", [G.PROP_RW, G.PROP_MLP, G.PROP_RW_POP, G.PROP_LANGEVIN])
def test_sampler_reaches_the_exact_posterior(proposal):
    w = W.preset("lingauss", proposal=proposal)
    y = W.observations(w)
    gm, gsd = grid_posterior(w, y)
    R = 8
    runs = [dict(T=w["T"], nx=w["nx"], seed=s, y=y) for s in range(1, R + 1)]
    _log("linear-Gaussian SMC^2, proposal %d: %d runs, N=%d, N_x=%d, K=%d" % (proposal, R, w["N"], w["nx"], w["K"]))
    smp = G.Sampler(w, runs)
    for _ in range(w["K"]):
        smp.step()
    est = np.array([smp.estimate(r)[0] for r in range(R)])
    sds = np.array([np.sqrt(np.diag(smp.estimate(r)[1])) for r in range(R)])
    rec = smp.records(0)
    smp.close()
    se = est.std(0, ddof=1) / np.sqrt(R)
    _log("  posterior mean %s (exact %s, s.e. %s); sd %s (exact %s); iterations by proposal code %s"
         % (est.mean(0), gm, se, sds.mean(0), gsd, np.bincount(rec[:, -2].astype(int), minlength=4).tolist()))
    if proposal in (G.PROP_RW_POP, G.PROP_LANGEVIN):
        assert np.all(rec[1:, -2] == (3 if proposal == G.PROP_RW_POP else 2))
    assert np.all(np.abs(est.mean(0) - gm) < 4 * se + 0.05 * gsd)
    assert np.all(np.abs(sds.mean(0) / gsd - 1) < 0.2)
