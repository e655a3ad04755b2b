"""The paper's SIR experiment and its printed SMC^2 estimates (tests/golden), shared
by the oracle test and the GPU test."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DATA_SEEDS = (2311, 1, 2, 3)  # synthetic observation series (the paper's are not published)


def load():
    vals = {}
    with open(os.path.join(HERE, "golden", "paper_sir_results.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def check(means, sds, g):
    """means, sds: [runs][2] recycled posterior means and standard deviations of
    (beta, gamma). Each run's mean lies within 3 posterior standard deviations of the
    truth; averaged over the runs, the means agree with the paper's to within 0.02
    (beta) and 0.005 (gamma), and the mean squared error is within a factor 10 of the
    paper's (the runs see different synthetic data, so only the order is comparable)."""
    truth = np.array([g["truth_beta"], g["truth_gamma"]])
    means, sds = np.asarray(means), np.asarray(sds)
    assert np.all(np.abs(means - truth) <= 3 * sds), (means, sds)
    avg = means.mean(axis=0)
    assert abs(avg[0] - g["smc2_mean_beta"]) <= 0.02, avg
    assert abs(avg[1] - g["smc2_mean_gamma"]) <= 0.005, avg
    mse = float(np.mean((means - truth) ** 2))
    assert mse <= 10 * g["smc2_mse"], mse
    return avg, mse
