"""The no-allocation particle-filter entry point (smc2_pf_loglik_noalloc) against the
workspace entry point (smc2_pf_loglik), through the C ABI.

Both run the same filter kernels on the same inputs, so their log-likelihoods are
identical. Calls in a row, the second with a smaller run (fewer filters, fewer days,
fewer particles), show that the static scratch keeps no state that matters between
calls; a third on the age-structured model stages four observation series."""
import numpy as np
import pytest

import paper_2311_12973_amd as G
from paper_2311_12973_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(name, n_theta, T, seed):
    w = dict(W.preset(name), T=T)
    y = W.observations(w)
    rng = np.random.default_rng(seed)
    theta = np.array(w["truth"]) * np.exp(rng.normal(0, 0.15, size=(n_theta, w["D"])))
    theta[:, 3] = np.clip(theta[:, 3], 1e-7, 1e-3)
    return w, y, theta


def test_noalloc_matches_workspace_entry_point_on_calls_in_a_row():
    for name, n_theta, T, nx, seed in [("seir", 96, 100, 256, 1), ("seir", 24, 37, 128, 2), ("age_seir", 16, 45, 96, 3)]:
        print("noalloc case %s n=%d T=%d nx=%d" % (name, n_theta, T, nx), flush=True)
        w, y, theta = _case(name, n_theta, T, seed)
        want = G.pf_loglik(w, theta, y, nx, seed=5, k=3)
        got = G.pf_loglik_noalloc(w, theta, y, nx, seed=5, k=3)
        assert np.isfinite(want).sum() >= n_theta // 2
        assert np.array_equal(np.isfinite(got), np.isfinite(want))
        assert np.array_equal(got, want), (name, np.abs(got - want).max())


def test_noalloc_rejects_a_run_beyond_the_static_scratch():
    w, y, theta = _case("seir", 4, 100, 4)
    yl = np.tile(y, (11, 1))[:1100]
    with pytest.raises(G.Smc2Error):
        G.pf_loglik_noalloc(w, theta, yl, 64, seed=5, k=3)
