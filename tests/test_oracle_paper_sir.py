"""Pin of the oracle's whole sampler against the paper's SIR experiment (Sec. V-A/V-B,
Table II): with the paper's model, priors, proposal and sizes, SMC^2 recovers the true
parameters to the accuracy the paper reports. A biased weight (a dropped L-kernel term,
a sign error in a log density, a wrong recycling weight) moves the means by several
posterior standard deviations. Four synthetic datasets, about 15 s on the CPU."""
import numpy as np

import oracle as O
from paper_2311_12973_amd import workloads as W
from tests import paper_sir_golden as PG


def test_oracle_recovers_the_papers_sir_estimates():
    g = PG.load()
    w = W.preset("paper_sir")
    assert w["truth"] == [g["truth_beta"], g["truth_gamma"]] and w["T"] == g["T"] and w["n_pop"] == g["n_pop"]
    assert (w["N"], w["K"], w["nx"]) == (g["N"], g["K"], g["N_x"]) and w["fixed"] == [g["initially_infected"]]
    assert np.allclose(w["rw_cov"], g["rw_sigma"] * np.eye(2))
    cfg = O.config_from_workload(w)
    means, sds = [], []
    for ds in PG.DATA_SEEDS:
        y = W.observations(dict(w, data_seed=ds))
        out = O.smc2_run(cfg, y, w["nx"], w["seed"], w["N"], w["K"])
        m, c, _ = O.recycle(out["rec"], 2)
        means.append(m)
        sds.append(np.sqrt(np.diag(c)))
    avg, mse = PG.check(means, sds, g)
    print("mean over datasets", avg, "mse %.3g" % mse)
