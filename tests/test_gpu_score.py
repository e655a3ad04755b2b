"""The GPU score estimator (smc2_pf_score) against the reference and against exact
gradients, through the C ABI.

* The score launch runs the same filter: its log-likelihoods equal the per-draw
  schedule's bit for bit.
* Parity with the reference score (or_pf_score, or_pf_lg) on the same streams, for SIR
  (both observation models), SEIR with r fixed and estimated, FP32 and FP64 filters, the
  linear-Gaussian model, ragged N_x and several workgroup sizes. Both sides take the same
  integer decisions and form the same FP64 terms; they differ only in the summation order
  of the final weighted mean (chunks of 64 particles on the GPU).
* Direct pins on the GPU: at N_x = 2048 (the score launch's limit) the mean over 400 GPU
  filters equals the exact gradient (central differences of the Kalman log-likelihood,
  and of the enumerated likelihood of a tiny SEIR population with r estimated) within
  four standard errors and a small allowance for the estimator's O(1/N_x) bias. (The
  tiny SIR problem of the reference's pin needs larger N_x: its bias at 2048 particles is
  1.4% of the gradient.)
* A filter whose weights vanish gets -inf and a zero score.
* The pooled score launch (the default where it fits) equals the per-draw one bit for
  bit, with and without resampling every day.
"""
import numpy as np
import pytest

import oracle as O
import paper_2311_12973_amd as G
from paper_2311_12973_amd import workloads as W
from tests import exact_models as X
from tests.test_oracle_score import central_difference

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def _theta(w, n, seed=3):
    rng = np.random.default_rng(seed)
    th = np.array(w["truth"]) * np.exp(rng.normal(0, 0.1, size=(n, w["D"])))
    if w["model"] == W.SEIR:
        th[:, 3] = np.clip(th[:, 3], 1e-7, 1e-3)
    return th


def _compare(got, ref):
    """relative to the scale of the coordinate over the batch (the weighted means can
    cancel to near zero, where a relative error means little)"""
    scale = np.maximum(1.0, np.abs(ref).max(axis=0))
    return float((np.abs(got - ref) / scale).max())


CASES = [  # workload, overrides, precision, nx, T, block
    ("sir_fp64", {}, G.PREC_FP64, 64, None, 0),
    ("sir_fp64", {"obs": W.OBS_POIS_PREV}, G.PREC_FP64, 100, None, 64),
    ("sir_fp64", {}, G.PREC_FP32, 257, None, 128),
    ("seir", {}, G.PREC_FP32, 512, 60, 0),
    ("seir", {}, G.PREC_FP64, 300, 40, 1024),
    ("seir_learned", {}, G.PREC_FP32, 1000, 50, 256),
    ("seir_learned", {}, G.PREC_FP64, 1, 30, 0),
    ("sir_fp64", {"pf_resampling": G.PF_RS_MULTINOMIAL}, G.PREC_FP64, 100, None, 0),
    ("seir", {"pf_resampling": G.PF_RS_MULTINOMIAL, "pf_always": 1}, G.PREC_FP32, 300, 40, 256),
]


@pytest.mark.parametrize("name,over,prec,nx,T,block", CASES)
def test_score_matches_reference(name, over, prec, nx, T, block):
    w = W.preset(name, **over)
    if T is not None:
        w["T"] = T
    y = W.observations(w)
    th = _theta(w, 12)
    _log("score %s %s prec=%d nx=%d block=%d" % (name, over, prec, nx, block))
    ll, sc = G.pf_score(w, th, y, nx, 9, 2, precision=prec, block=block)
    ll_pd = G.pf_loglik(w, th, y, nx, 9, 2, precision=prec, block=block, schedule=G.SCHED_PER_DRAW)
    assert np.array_equal(ll, ll_pd)
    cfg = O.config_from_workload(w, prec=prec)
    ref = [O.pf_score(cfg, th[i], y, nx, 9, i, 2) for i in range(len(th))]
    ll_ref = np.array([r[0] for r in ref])
    sc_ref = np.array([r[1] for r in ref])
    fin = np.isfinite(ll_ref)
    assert fin.sum() >= len(th) // 2
    assert np.array_equal(np.isfinite(ll), fin)
    assert np.allclose(ll[fin], ll_ref[fin], rtol=1e-12 if prec == G.PREC_FP64 else 1e-4, atol=0)
    err = _compare(sc[fin], sc_ref[fin])
    _log("  score max error %.3g (of each coordinate's scale)" % err)
    assert err <= 1e-9
    assert np.all(sc[~fin] == 0.0)
    if w["model"] == W.SEIR:
        assert np.all(sc[:, 3] == 0.0)


POOLED_CASES = [  # workload, overrides, precision, nx, T, block, resample every day
    ("sir_fp64", {}, G.PREC_FP64, 100, None, 0, 0),
    ("sir_fp64", {"obs": W.OBS_POIS_PREV}, G.PREC_FP32, 257, None, 128, 1),
    ("seir", {}, G.PREC_FP32, 512, 60, 0, 0),
    ("seir", {}, G.PREC_FP32, 1000, 40, 1024, 1),
    ("seir", {}, G.PREC_FP64, 300, 40, 256, 0),
    ("seir_learned", {}, G.PREC_FP32, 1024, 50, 0, 0),
    ("seir_learned", {}, G.PREC_FP64, 65, 30, 64, 1),
]


@pytest.mark.parametrize("name,over,prec,nx,T,block,always", POOLED_CASES)
def test_pooled_score_launch_equals_the_per_draw_one(name, over, prec, nx, T, block, always):
    """The pooled draw schedule adds each day's score terms when it applies the drawn
    flows, from the day-start counts, in the per-draw schedule's order: the same bits."""
    w = W.preset(name, **over)
    if T is not None:
        w["T"] = T
    y = W.observations(w)
    th = _theta(w, 16, seed=5)
    _log("pooled score %s %s prec=%d nx=%d block=%d always=%d" % (name, over, prec, nx, block, always))
    ll_p, sc_p = G.pf_score(w, th, y, nx, 4, 3, precision=prec, block=block, pf_always=always,
                            schedule=G.SCHED_POOLED)
    ll_d, sc_d = G.pf_score(w, th, y, nx, 4, 3, precision=prec, block=block, pf_always=always,
                            schedule=G.SCHED_PER_DRAW)
    assert np.isfinite(ll_d).sum() >= len(th) // 2
    assert np.array_equal(ll_p, ll_d)
    assert np.array_equal(sc_p, sc_d)
    ll_a, sc_a = G.pf_score(w, th, y, nx, 4, 3, precision=prec, block=block, pf_always=always)
    assert np.array_equal(ll_a, ll_d) and np.array_equal(sc_a, sc_d)


@pytest.mark.parametrize("nx,k,block", [(64, 0, 0), (1000, 3, 256), (2048, 5, 0)])
def test_linear_gaussian_score_matches_reference(nx, k, block):
    w = W.preset("lingauss")
    y = W.simulate(W.LINGAUSS, W.OBS_GAUSS, 1.0, [0.9, 1.0, 1.0], 60, 23, w["fixed"])
    th = np.array([[0.9, 1.0, 1.0], [0.5, 0.3, 2.0], [-0.7, 1.5, 0.4], [0.99, 0.8, 1.1]])
    ll, sc = G.pf_score(w, th, y, nx, 17, k, block=block)
    ref = [O.pf_lg(t[0], t[1], t[2], w["fixed"][0], w["fixed"][1], y, nx, 17, filt=i, k=k, score=True)
           for i, t in enumerate(th)]
    assert np.allclose(ll, [r[0] for r in ref], rtol=1e-11, atol=1e-9)
    err = _compare(sc, np.array([r[1] for r in ref]))
    _log("linear-Gaussian score nx=%d: max error %.3g" % (nx, err))
    assert err <= 1e-9


def _close(sc, exact, rel_bias=0.005):
    mean, se = sc.mean(0), sc.std(0, ddof=1) / np.sqrt(len(sc))
    return np.all(np.abs(mean - exact) < 4 * se + rel_bias * np.maximum(1.0, np.abs(exact))), mean, se


def test_gpu_score_equals_the_kalman_gradient():
    from tests.test_oracle_kalman import M0, PHI, S0, SQ, SR, kalman_loglik, simulate
    y = simulate(25, 11)
    exact = central_difference(lambda v: kalman_loglik(v[0], v[1], v[2], M0, S0, y), [PHI, SQ, SR], 1e-5)
    w = W.preset("lingauss", fixed=[M0, S0])
    _, sc = G.pf_score(w, np.tile([PHI, SQ, SR], (400, 1)), y, 2048, 7, 1)
    ok, mean, se = _close(sc, exact)
    _log("GPU linear-Gaussian score %s (exact %s, s.e. %s)" % (mean, exact, se))
    assert ok


def test_gpu_score_equals_the_exact_seir_gradient():
    n_pop, T, r = 8, 5, 3.0
    beta, sigma, gamma = 1.6, 0.5, 0.3
    iota = 2.0 / n_pop
    y = W.simulate(W.SEIR, W.OBS_NB_INC, n_pop, [beta, sigma, gamma, iota], T, seed=21, fixed=[r], min_frac=0)
    exact = central_difference(lambda v: X.seir_loglik(v[0], v[1], v[2], n_pop, 2, y, v[3]), [beta, sigma, gamma, r])
    w = dict(W.preset("seir_learned"), n_pop=float(n_pop), prec=G.PREC_FP64)
    _, sc = G.pf_score(w, np.tile([beta, sigma, gamma, iota, r], (400, 1)), y, 2048, 3, 1)
    assert np.all(sc[:, 3] == 0.0)
    ok, mean, se = _close(sc[:, [0, 1, 2, 4]], exact)
    _log("GPU SEIR score %s (exact %s, s.e. %s)" % (mean, exact, se))
    assert ok


def test_dead_filter_has_zero_score():
    w = dict(W.preset("paper_sir"), fixed=[0])
    y = np.zeros((5, 1), dtype=np.int32)
    y[2, 0] = 3
    ll, sc = G.pf_score(w, np.array([[0.5, 0.2]] * 3), y, 64, 1, 1)
    assert np.all(ll == -np.inf) and np.all(sc == 0.0)
