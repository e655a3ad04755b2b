"""Event counts of the reference particle filter (the unit of work of the kernel's
roofline): the counts obey the structure of the method on a small SEIR filter."""
import numpy as np

import oracle as O
from oracle import opcount
from paper_2311_12973_amd import workloads as W


def test_event_counts_follow_the_method():
    w = W.preset("seir")
    cfg = O.config_from_workload(w)
    y = W.observations(w)[:30]
    nx, T = 96, 30
    O.events_reset()
    ll = O.pf_loglik(cfg, np.array(w["truth"]), y, nx, 5, 0, 1)
    ev = O.events_get()
    assert np.isfinite(ll)
    assert ev["pstep"] == nx * T
    assert ev["draw"] == 3 * ev["pstep"]  # S->E, E->I, I->R per particle-day
    assert ev["inv"] + ev["btrs"] <= ev["draw"]
    assert ev["btrs"] <= ev["attempt"] and ev["final"] <= ev["attempt"]
    # one Philox call per inversion, one per two BTRS attempts (rounded up per draw)
    assert ev["btrs"] <= ev["philox"] - ev["inv"] <= ev["attempt"]
    assert ev["philox"] - ev["inv"] >= ev["attempt"] / 2
    # FP64 transcendentals: hazard (1) + NB observation (2) + weight (1) per particle-step,
    # two per inversion, six per final test
    assert ev["t64"] == 4 * ev["pstep"] + 2 * ev["inv"] + 6 * ev["final"]
    assert ev["rs_particle"] % nx == 0 and ev["rs_particle"] <= nx * (T - 1)
    # a second filter adds to the totals; a reset clears them
    O.pf_loglik(cfg, np.array(w["truth"]), y, nx, 5, 1, 1)
    assert O.events_get()["pstep"] == 2 * nx * T
    O.events_reset()
    assert O.events_get()["pstep"] == 0


def test_operation_count_is_the_priced_sum():
    r = opcount.count(dict(W.preset("seir"), T=20), N=8, K=2, nx=64)
    per = r["per_pstep"]
    assert per["pstep"] == 1.0
    assert r["ops_per_pstep"] == sum(opcount.COST[k] * per[k] for k in opcount.COST)
    assert 300 < r["ops_per_pstep"] < 2000
