"""The FP64 replay of a filter from injected integer decisions (or_pf_replay), the
reference's half of the precision report: given a trajectory's per-day counts,
ancestors and resampling flags it recomputes the likelihood estimate in FP64 (Sec. II
weights, increments and mean-weight reset).

* Replaying the FP64 reference filter's own decisions reproduces its estimate and
  every increment exactly (the same FP64 operations on the same counts), for every
  model and observation, adaptive and every-step resampling, systematic and
  multinomial ancestors (which the observed new cases depend on after a resampling).
* Wrong ancestors or a wrong flag change the result.
* Replaying the FP32 filter's decisions gives an estimate within FP32 weight rounding
  of the FP32 filter's own (the per-step weight error of the FP32 path).
"""
import numpy as np
import pytest

import oracle as O
from paper_2311_12973_amd import workloads as W

CASES = [("sir_fp64", O.OBS_POIS_INC, 64, 30), ("paper_sir", O.OBS_POIS_PREV, 100, 30),
         ("seir", O.OBS_NB_INC, 128, 60), ("age_seir", O.OBS_NB_INC, 64, 50)]


def _case(name, T):
    w = dict(W.preset(name), T=T)
    y = W.observations(w)
    rng = np.random.default_rng(3)
    theta = np.array(w["truth"]) * np.exp(rng.normal(0, 0.1, size=(6, w["D"])))
    if w["model"] != O.SIR:
        theta[:, 3] = np.clip(theta[:, 3], 1e-7, 1e-3)
    return w, y, theta


@pytest.mark.parametrize("pf_always,resampling", [(0, O.RS_SYSTEMATIC), (1, O.RS_SYSTEMATIC),
                                                  (1, O.RS_MULTINOMIAL)])
@pytest.mark.parametrize("name,obs,nx,T", CASES)
def test_replay_of_the_fp64_filter_is_exact(name, obs, nx, T, pf_always, resampling):
    w, y, theta = _case(name, T)
    w = dict(w, pf_always=pf_always, pf_resampling=resampling)
    cfg = O.config_from_workload(w, prec=O.PREC_FP64)
    resampled = 0
    for i, th in enumerate(theta):
        ll, inc, rs, st, anc = O.pf_trace_full(cfg, th, y, nx, 5, i, 2)
        resampled += rs.sum()
        ll2, inc2 = O.pf_replay(cfg, th, y, st, anc, rs)
        assert ll2 == ll or (ll == -np.inf and ll2 == -np.inf), (i, ll, ll2)
        assert np.array_equal(inc2, inc)
    assert resampled > 0


def test_replay_depends_on_the_injected_ancestors_and_flags():
    w, y, theta = _case("seir", 60)
    cfg = O.config_from_workload(w, prec=O.PREC_FP64)
    ll, inc, rs, st, anc = O.pf_trace_full(cfg, theta[0], y, 128, 5, 0, 2)
    t = int(np.flatnonzero(rs)[0])
    bad = anc.copy()
    bad[t] = np.roll(bad[t], 1)
    assert O.pf_replay(cfg, theta[0], y, st, bad, rs)[0] != ll
    rs2 = rs.copy()
    rs2[t] = 0
    assert O.pf_replay(cfg, theta[0], y, st, anc, rs2)[0] != ll


@pytest.mark.parametrize("name,obs,nx,T", CASES[2:])
def test_replay_of_the_fp32_filter_measures_its_weight_rounding(name, obs, nx, T):
    w, y, theta = _case(name, T)
    cfg32 = O.config_from_workload(w, prec=O.PREC_FP32)
    cfg64 = O.config_from_workload(w, prec=O.PREC_FP64)
    for i, th in enumerate(theta):
        ll, inc, rs, st, anc = O.pf_trace_full(cfg32, th, y, nx, 5, i, 2)
        ll64, _ = O.pf_replay(cfg64, th, y, st, anc, rs)
        assert np.isfinite(ll) and abs(ll64 - ll) <= 1e-5 * abs(ll), (i, ll, ll64)
