"""GPU parity of the building blocks against the CPU reference (through the C ABI).

* Philox words: bit-exact.
* Binomial draws (FP32 and FP64 sampler, inversion and BTRS regimes): identical
  integers at the same (n, p, counter coordinates).
* Integer systematic resampling: identical ancestors and ESS decisions for the same
  quantised weights and 64-bit uniform, including ragged sizes.
* Particle-filter log-likelihoods: FP64 within 1e-12 relative, FP32 within the 1e-4
  relative tolerance of the FP32 path (identical integer decisions give ~1e-12), for
  several workgroup sizes (results must not depend on the tiling).
"""
import numpy as np
import pytest

import oracle as O
import paper_2311_12973_amd as G
from paper_2311_12973_amd import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def test_philox_bit_exact():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    for seed in [0, 1, 0xDEADBEEFCAFEBABE]:
        got = G.philox_batch(ctr, seed)
        key = [seed & 0xFFFFFFFF, seed >> 32]
        for e in range(0, 4096, 7):
            assert np.array_equal(got[e], O.philox(ctr[e], key)), (seed, e)


CELLS = [(0, 0.3), (1, 0.3), (17, 0.0), (17, 1.0), (5, 0.5), (30, 0.2), (30, 0.9), (100, 0.099), (100, 0.101),
         (1000, 1e-3), (1000, 0.5), (1000, 0.97), (40000, 0.0003), (40000, 0.2), (10**6, 1e-6), (10**6, 2e-5),
         (10**6, 0.003), (10**6, 0.22), (10**6, 0.5), (250000, 0.6), (16777216, 0.01)]


@pytest.mark.parametrize("prec", [G.PREC_FP64, G.PREC_FP32])
def test_binomial_bit_exact(prec):
    count = 4096
    total = 0
    for (n, p) in CELLS:
        _log("binomial prec=%d n=%d p=%g" % (prec, n, p))
        p_eff = float(np.float32(p)) if prec == G.PREC_FP32 else p
        got = G.binomial_batch(prec, np.full(count, n), np.full(count, p_eff), seed=77, i=5, k=3, t=11, b=2)
        want = O.binomial_batch(prec, n, p_eff, 77, count, i=5, k=3, t=11, b=2)
        mism = np.flatnonzero(got != want)
        assert len(mism) == 0, (n, p, mism[:10], got[mism[:10]], want[mism[:10]])
        total += count
    # heterogeneous lanes in one launch (divergent regimes inside a wave)
    rng = np.random.default_rng(9)
    n = rng.integers(0, 200000, size=8192)
    p = rng.random(8192) ** 3
    if prec == G.PREC_FP32:
        p = p.astype(np.float32).astype(np.float64)
    got = G.binomial_batch(prec, n, p, seed=3, i=1, k=1, t=1, b=0)
    want = np.array([O.binomial(prec, n[j], p[j], 3, j, 1, 1, 1, 0) for j in range(len(n))])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("prec", [G.PREC_FP64, G.PREC_FP32])
def test_binomial_bit_exact_many(prec):
    """About a million draws over random (n, p) in both regimes: rare rounding
    differences (an FP32 operation that is not correctly rounded, a fused
    multiply-add) show up here."""
    rng = np.random.default_rng(17 + prec)
    M = 1 << 20
    n = np.floor(10 ** rng.uniform(0, 6.3, M)).astype(np.int32)
    p = 10 ** rng.uniform(-6, np.log10(0.95), M)
    if prec == G.PREC_FP32:
        p = p.astype(np.float32).astype(np.float64)
    got = G.binomial_batch(prec, n, p, seed=123, i=7, k=4, t=33, b=1)
    want = O.binomial_many(prec, n, p, 123, i=7, k=4, t=33, b=1)
    bad = np.flatnonzero(got != want)
    assert len(bad) == 0, [(int(n[j]), float(p[j]), int(got[j]), int(want[j])) for j in bad[:8]]


def test_binomial_btrs_final_test_decisions():
    """Four million FP32 draws in the transformed-rejection regime (n p >= 10), where
    about a third of the attempts reach the final acceptance test: the kernels decide
    it in FP32 with an error bound and fall back to FP64 near the boundary, and every
    draw must equal the reference's (which always takes the FP64 test). The sizes
    cover both sides of n = 2^23, above which the FP64 test always decides."""
    rng = np.random.default_rng(2311)
    M = 1 << 22
    n = np.floor(10 ** rng.uniform(1.3, 7.4, M)).astype(np.int64)
    n[: M // 16] = rng.integers((1 << 23) - 4096, (1 << 23) + 4096, M // 16)
    n = np.minimum(n, (1 << 31) - 1).astype(np.int32)
    lo = np.log10(10.0 / n)
    p = 10 ** (lo + (np.log10(0.5) - lo) * rng.random(M))
    p = p.astype(np.float32).astype(np.float64)
    got = G.binomial_batch(G.PREC_FP32, n, p, seed=99, i=3, k=2, t=17, b=0)
    want = O.binomial_many(G.PREC_FP32, n, p, 99, i=3, k=2, t=17, b=0)
    bad = np.flatnonzero(got != want)
    assert len(bad) == 0, [(int(n[j]), float(p[j]), int(got[j]), int(want[j])) for j in bad[:8]]


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 257, 500, 1000, 2048, 4096])
def test_resample_bit_exact(n):
    rng = np.random.default_rng(n)
    S = 24
    q = np.zeros((S, n), dtype=np.uint64)
    for s in range(S):
        kind = s % 4
        if kind == 0:
            w = rng.random(n)
        elif kind == 1:
            w = np.exp(rng.normal(0, 5, n))
        elif kind == 2:
            w = np.where(rng.random(n) < 0.05, rng.random(n), 0.0)
            w[rng.integers(n)] = 1.0
        else:
            w = np.ones(n)
        q[s] = np.floor(w / w.max() * 2.0**32).astype(np.uint64)
    x64 = rng.integers(0, 2**63, size=S, dtype=np.uint64) * np.uint64(2)
    x64[0] = 0
    x64[1] = np.uint64(2**64 - 1)
    anc, trig = G.resample_batch(q, x64)
    for s in range(S):
        assert np.array_equal(anc[s], O.resample_ancestors(q[s], int(x64[s]))), s
        assert bool(trig[s]) == O.resample_trigger(q[s]), s


def _pf_case(name, prec, nx, n_theta, T=None, pf_always=0, seed=11, k=2):
    w = W.preset(name)
    if T is not None:
        w["T"] = T
    y = W.observations(w)
    rng = np.random.default_rng(seed)
    truth = np.array(w["truth"])
    theta = truth * np.exp(rng.normal(0, 0.15, size=(n_theta, w["D"])))
    if w["model"] in (W.SEIR, W.AGE_SEIR):
        theta[:, 3] = np.clip(theta[:, 3], 1e-7, 1e-3)
    return w, y, theta


_PF_CASES = [("sir_fp64", G.PREC_FP64, 64, None), ("sir_fp64", G.PREC_FP32, 100, None),
             ("paper_sir", G.PREC_FP64, 500, None), ("seir", G.PREC_FP32, 512, 60), ("seir", G.PREC_FP64, 300, 40),
             ("age_seir", G.PREC_FP32, 300, 60), ("age_seir", G.PREC_FP64, 130, 40)]


# the pooled schedule covers SIR and SEIR; the age-structured model always runs per draw
@pytest.mark.parametrize("name,prec,nx,T,schedule",
                         [c + (G.SCHED_PER_DRAW,) for c in _PF_CASES] +
                         [c + (G.SCHED_POOLED,) for c in _PF_CASES if c[0] != "age_seir"])
@pytest.mark.parametrize("block", [0, 64, 128, 512])
def test_pf_loglik_matches_oracle(name, prec, nx, T, block, schedule):
    _log("pf %s prec=%d nx=%d block=%d schedule=%d" % (name, prec, nx, block, schedule))
    w, y, theta = _pf_case(name, prec, nx, 24, T)
    got = G.pf_loglik(w, theta, y, nx, seed=9, k=2, precision=prec, block=block, schedule=schedule)
    cfg = O.config_from_workload(w, prec=prec)
    want = np.array([O.pf_loglik(cfg, theta[i], y, nx, 9, i, 2) for i in range(len(theta))])
    fin = np.isfinite(want)
    assert np.array_equal(np.isfinite(got), fin)
    rel = np.abs(got[fin] - want[fin]) / np.abs(want[fin])
    _log("  max rel err %.3g" % rel.max())
    assert rel.max() <= (1e-12 if prec == G.PREC_FP64 else 1e-4)
    # identical integer decisions leave only FP64 summation-order noise
    assert np.mean(rel < 1e-11) >= 0.95


@pytest.mark.parametrize("schedule", [G.SCHED_PER_DRAW, G.SCHED_POOLED])
def test_pf_resample_every_step_and_ragged(schedule):
    w = W.preset("sir_fp64")
    y = W.observations(w)
    theta = np.array([w["truth"]] * 10) * np.linspace(0.8, 1.2, 10)[:, None]
    for nx in [1, 7, 65, 129]:
        got = G.pf_loglik(w, theta, y, nx, seed=4, k=1, pf_always=1, schedule=schedule)
        cfg = O.config_from_workload(w)
        cfg.pf_always = 1
        want = np.array([O.pf_loglik(cfg, theta[i], y, nx, 4, i, 1) for i in range(10)])
        fin = np.isfinite(want)
        assert np.array_equal(np.isfinite(got), fin)
        assert np.allclose(got[fin], want[fin], rtol=1e-12, atol=0)


@pytest.mark.parametrize("name,prec,nx,T", [("sir_fp64", G.PREC_FP64, 129, None), ("seir", G.PREC_FP32, 512, 60),
                                            ("seir", G.PREC_FP64, 200, 30), ("age_seir", G.PREC_FP32, 300, 40)])
@pytest.mark.parametrize("pf_always", [0, 1])
def test_pf_multinomial_resampling_matches_oracle(name, prec, nx, T, pf_always):
    """Multinomial resampling (one uniform per slot): log-likelihoods against the
    reference, and every day's counts of two filters bit-identical to the reference's
    (the ancestors are identical)."""
    _log("pf multinomial %s prec=%d nx=%d pf_always=%d" % (name, prec, nx, pf_always))
    w, y, theta = _pf_case(name, prec, nx, 16, T)
    w = dict(w, pf_resampling=G.PF_RS_MULTINOMIAL)
    got = G.pf_loglik(w, theta, y, nx, seed=9, k=2, precision=prec, pf_always=pf_always)
    cfg = O.config_from_workload(w, prec=prec)
    cfg.pf_always = pf_always
    want = np.array([O.pf_loglik(cfg, theta[i], y, nx, 9, i, 2) for i in range(len(theta))])
    fin = np.isfinite(want)
    assert np.array_equal(np.isfinite(got), fin)
    rel = np.abs(got[fin] - want[fin]) / np.abs(want[fin])
    assert rel.max() <= (1e-12 if prec == G.PREC_FP64 else 1e-4)
    assert np.mean(rel < 1e-11) >= 0.95
    sys_ll = G.pf_loglik(dict(w, pf_resampling=G.PF_RS_SYSTEMATIC), theta, y, nx, seed=9, k=2, precision=prec,
                         pf_always=pf_always)
    assert not np.array_equal(got, sys_ll)
    if pf_always:
        _, _, rs, st = G.pf_trace_state(dict(w, pf_always=1), theta[:2], y, nx, seed=9, k=2, precision=prec)
        for i in range(2):
            _, _, rs_ref, st_ref = O.pf_trace_state(cfg, theta[i], y, nx, 9, i, 2)
            assert np.array_equal(rs[i], rs_ref)
            assert np.array_equal(st[i], st_ref)


@pytest.mark.parametrize("name,prec,nx,T", [("seir", G.PREC_FP32, 4096, 20), ("sir_fp64", G.PREC_FP64, 4096, 30),
                                            ("age_seir", G.PREC_FP32, 2048, 12)])
@pytest.mark.parametrize("block", [0, 1024])
@pytest.mark.parametrize("schedule", [G.SCHED_AUTO, G.SCHED_PER_DRAW])
def test_pf_maximum_particles_matches_oracle(name, prec, nx, T, block, schedule):
    """The largest particle count the interface accepts per model (4096; 2048 for the
    age model), with the automatic and the per-draw schedule, against the reference."""
    _log("pf max %s prec=%d nx=%d block=%d schedule=%d" % (name, prec, nx, block, schedule))
    w, y, theta = _pf_case(name, prec, nx, 8, T)
    got = G.pf_loglik(w, theta, y, nx, seed=5, k=3, precision=prec, block=block, schedule=schedule)
    cfg = O.config_from_workload(w, prec=prec)
    want = np.array([O.pf_loglik(cfg, theta[i], y, nx, 5, i, 3) for i in range(len(theta))])
    fin = np.isfinite(want)
    assert fin.sum() >= 4
    assert np.array_equal(np.isfinite(got), fin)
    rel = np.abs(got[fin] - want[fin]) / np.abs(want[fin])
    _log("  max rel err %.3g" % rel.max())
    assert rel.max() <= (1e-12 if prec == G.PREC_FP64 else 1e-4)


def test_pf_dead_filter_is_minus_inf():
    w = W.preset("paper_sir")
    y = np.zeros((5, 1), dtype=np.int32)
    y[2, 0] = 3
    w = dict(w, fixed=[0])  # nobody infected: Poisson(I_t = 0) cannot produce y = 3
    ll = G.pf_loglik(w, np.array([[0.5, 0.2]] * 3), y, 64, seed=1, k=1)
    assert np.all(ll == -np.inf)


@pytest.mark.parametrize("name,prec,nx,T", [("seir", G.PREC_FP32, 512, 100), ("seir", G.PREC_FP64, 512, 100),
                                            ("paper_sir", G.PREC_FP64, 500, 30), ("sir_fp64", G.PREC_FP32, 300, 50)])
def test_pf_schedules_identical(name, prec, nx, T):
    """The pooled schedule (final acceptance tests batched per wave) and the per-draw
    schedule draw identical flows, so the log-likelihoods and the per-day states agree
    to the last bit, here at the benchmark's filter shape."""
    _log("schedules %s prec=%d nx=%d T=%d" % (name, prec, nx, T))
    w, y, theta = _pf_case(name, prec, nx, 64, T)
    a = G.pf_loglik(w, theta, y, nx, seed=21, k=3, precision=prec, schedule=G.SCHED_PER_DRAW)
    b = G.pf_loglik(w, theta, y, nx, seed=21, k=3, precision=prec, schedule=G.SCHED_POOLED)
    assert np.array_equal(a, b)
    sa = G.pf_trace_state(w, theta[:4], y, nx, seed=21, k=3, precision=prec, schedule=G.SCHED_PER_DRAW)
    sb = G.pf_trace_state(w, theta[:4], y, nx, seed=21, k=3, precision=prec, schedule=G.SCHED_POOLED)
    assert len(sa) == len(sb)
    for xa, xb in zip(sa, sb):
        assert np.array_equal(xa, xb)


def test_pf_results_do_not_depend_on_the_launch_round():
    """A launch whose filters are all resident at once sets the waves' issue priority
    from each filter's remaining work; a larger launch (several rounds of workgroups)
    leaves it alone. Priorities only order instruction issue, so the same filters give
    the same log-likelihoods to the last bit in both launches."""
    w, y, theta = _pf_case("seir", G.PREC_FP32, 512, 3000, T=40)
    small = G.pf_loglik(w, theta[:200], y, 512, seed=5, k=2, block=256)
    large = G.pf_loglik(w, theta, y, 512, seed=5, k=2, block=256)
    _log("single round %d filters, several rounds %d filters" % (200, len(theta)))
    assert np.isfinite(small).all()
    assert np.array_equal(small, large[:200])


@pytest.mark.parametrize("pf_always,resampling", [(1, G.PF_RS_SYSTEMATIC), (0, G.PF_RS_SYSTEMATIC),
                                                 (1, G.PF_RS_MULTINOMIAL)])
def test_pf_repeated_launches_are_identical(pf_always, resampling):
    """Every draw is a function of its coordinates, whichever wave takes it, so repeated
    launches at the benchmark's filter shape give identical log-likelihoods. Resampling
    every day puts a resampling gather before each day's draws: a missing barrier
    between the two let a wave read counts that another wave had not yet written back,
    and about one filter in a thousand then differed from launch to launch."""
    w, y, theta = _pf_case("seir", G.PREC_FP32, 512, 1024, T=100)
    w = dict(w, pf_resampling=resampling)
    ref = G.pf_loglik(w, theta, y, 512, seed=3, k=2, pf_always=pf_always)
    assert np.isfinite(ref).all()
    for rep in range(8):
        ll = G.pf_loglik(w, theta, y, 512, seed=3, k=2, pf_always=pf_always)
        _log("repeat %d: %d filters differ" % (rep, int((ll != ref).sum())))
        assert np.array_equal(ll, ref), (rep, np.flatnonzero(ll != ref)[:5])


def test_pooled_schedule_rejected_for_age_model():
    w = W.preset("age_seir")
    w["T"] = 5
    y = W.observations(w)
    with pytest.raises(RuntimeError):
        G.pf_loglik(w, np.array([w["truth"]] * 2), y, 64, seed=1, k=1, schedule=G.SCHED_POOLED)


@pytest.mark.parametrize("prec", [G.PREC_FP64, G.PREC_FP32])
def test_pf_age_seir_unequal_groups_matches_oracle(prec):
    """The age model's force of infection with unequal groups and a non-symmetric contact
    matrix: the enumerable four-group population of the reference's exact pin (sizes 3,
    3, 2, 2), and a large population with group fractions 0.4, 0.3, 0.2, 0.1 (the
    workloads use equal groups, where N_g and N_h coincide)."""
    from tests.test_oracle_pf_exact import AGE_THETA, age_pin_case
    cfg_small, y_small, _ = age_pin_case(prec)
    wa = W.preset("age_seir")
    fixed = list(np.asarray(wa["fixed"][:16])) + [0.4, 0.3, 0.2, 0.1]
    cases = [(dict(wa, n_pop=float(sum([3, 3, 2, 2])), fixed=[cfg_small.fixed[i] for i in range(20)]), y_small,
              np.tile(AGE_THETA, (64, 1)) * np.exp(np.random.default_rng(1).normal(0, 0.1, (64, 8))), 32),
             (dict(wa, fixed=fixed, T=60), None, None, 256)]
    for w, y, theta, nx in cases:
        if y is None:
            y = W.observations(w)
            rng = np.random.default_rng(2)
            theta = np.array(w["truth"]) * np.exp(rng.normal(0, 0.15, size=(24, 8)))
            theta[:, 3] = np.clip(theta[:, 3], 1e-7, 1e-3)
        _log("age unequal groups n_pop=%g nx=%d prec=%d" % (w["n_pop"], nx, prec))
        got = G.pf_loglik(w, theta, y, nx, seed=13, k=2, precision=prec)
        cfg = O.config_from_workload(w, prec=prec)
        want = np.array([O.pf_loglik(cfg, theta[i], y, nx, 13, i, 2) for i in range(len(theta))])
        fin = np.isfinite(want)
        assert fin.sum() >= len(theta) // 2
        assert np.array_equal(np.isfinite(got), fin)
        rel = np.abs(got[fin] - want[fin]) / np.abs(want[fin])
        _log("  max rel err %.3g" % rel.max())
        assert rel.max() <= (1e-12 if prec == G.PREC_FP64 else 1e-4)
