"""Pins of the reference's outer SMC^2 step (Sec. IV).

* Cholesky and Gaussian log-densities against numpy / scipy.
* The approximately optimal L-kernel (Sec. IV-D): fitted moments against numpy's
  weighted mean / covariance, and the Schur-complement identity
  log N_2D(z) = log N_D(theta_k; mu_2, S22) + log L(theta_{k-1} | theta_k),
  which fails for a wrong conditional mean, covariance or transposed block.
* The forward L-kernel special case (Eq. aimplified_l_weights): with a symmetric RW
  proposal the weight update is exactly the ratio of targets.
* ESS / l_k closed forms, recycling constants (Sec. IV-C), prior densities, the RW
  proposal covariance, and outer resampling against the exact-rational systematic
  resampling of the paper's equations.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from tests.test_oracle_resample import paper_systematic


def _spd(rng, n):
    A = rng.normal(size=(n, n))
    return A @ A.T + 0.3 * np.eye(n)


def test_cholesky_and_mvn():
    rng = np.random.default_rng(0)
    for n in range(1, 9):
        S = _spd(rng, n)
        st, L = O.cholesky(S)
        assert st == 0
        assert np.allclose(L, np.linalg.cholesky(S), rtol=1e-12, atol=1e-12)
        x, mu = rng.normal(size=n), rng.normal(size=n)
        want = stats.multivariate_normal(mu, S).logpdf(x)
        assert O.mvn_logpdf_chol(x, mu, L) == pytest.approx(want, rel=1e-11)
    st, _ = O.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert st == -1
    st, _ = O.cholesky(np.zeros((3, 3)))
    assert st == -1


@pytest.mark.parametrize("D", [1, 2, 4, 5, 8])
def test_lkernel_fit_moments_and_schur_identity(D):
    rng = np.random.default_rng(D)
    N = 400
    phi = rng.normal(size=(N, D)) @ rng.normal(size=(D, D))
    phi_new = phi + 0.5 * rng.normal(size=(N, D)) @ rng.normal(size=(D, D)) + 0.3 * phi**2 / (1 + phi**2)
    omega = rng.random(N) ** 3
    omega /= omega.sum()
    st, mu, A, LS = O.lkernel_fit(phi, phi_new, omega)
    assert st == 0
    Z = np.hstack([phi, phi_new])
    mu_np = np.average(Z, axis=0, weights=omega)
    cov_np = np.cov(Z.T, aweights=omega, bias=True).reshape(2 * D, 2 * D)
    assert np.allclose(mu, mu_np, rtol=1e-12, atol=1e-12)
    joint = stats.multivariate_normal(mu_np, cov_np)
    marg = stats.multivariate_normal(mu_np[D:], cov_np[D:, D:])
    for i in range(0, N, 37):
        mean = mu[:D] + A @ (phi_new[i] - mu[D:])
        logL = O.mvn_logpdf_chol(phi[i], mean, LS)
        lhs = joint.logpdf(Z[i])
        rhs = marg.logpdf(phi_new[i]) + logL
        assert lhs == pytest.approx(rhs, rel=1e-9, abs=1e-9)


def test_lkernel_fit_degenerate_fails():
    phi = np.ones((50, 2))
    st, *_ = O.lkernel_fit(phi, phi.copy(), np.full(50, 1 / 50))
    assert st == -1


def _cfg(D, lkernel=O.L_GAUSS_OPT, rw=None, prior=None):
    rw = np.eye(D) * 0.04 if rw is None else rw
    prior = [[O.PRIOR_NORMAL, 0.0, 2.0]] * D if prior is None else prior
    return O.make_config(O.SEIR, O.OBS_NB_INC, D, O.PREC_FP64, 1e6, prior, rw, [10.0], lkernel=lkernel)


def test_prior_logpdf_and_transforms():
    cfg = O.make_config(O.SEIR, O.OBS_NB_INC, 4, O.PREC_FP64, 1e6,
                        [[O.PRIOR_LOGNORMAL, -0.9, 0.5], [O.PRIOR_UNIFORM, 0.1, 0.7],
                         [O.PRIOR_LOGITNORMAL, -11.5, 1.0], [O.PRIOR_NORMAL, 2.0, 3.0]], np.eye(4), [10])
    phi = np.array([-1.2, 0.4, -10.0, 0.5])
    want = (stats.norm(-0.9, 0.5).logpdf(-1.2) + stats.uniform(0.1, 0.6).logpdf(0.4)
            + stats.norm(-11.5, 1.0).logpdf(-10.0) + stats.norm(2.0, 3.0).logpdf(0.5))
    assert O.prior_logpdf(cfg, phi) == pytest.approx(want, rel=1e-13)
    assert O.prior_logpdf(cfg, np.array([-1.2, 0.75, -10.0, 0.5])) == -np.inf
    th = O.theta_of_phi(cfg, phi)
    assert th == pytest.approx([np.exp(-1.2), 0.4, 1 / (1 + np.exp(10.0)), 0.5], rel=1e-15)


def test_prior_draw_distribution():
    cfg = O.make_config(O.SIR, O.OBS_POIS_INC, 2, O.PREC_FP64, 1e4,
                        [[O.PRIOR_LOGNORMAL, -1.0, 0.5], [O.PRIOR_UNIFORM, 0.0, 1.0]], np.eye(2), [3])
    phi, lp = O.prior_draw(cfg, 20000, 7)
    assert stats.kstest(phi[:, 0], stats.norm(-1.0, 0.5).cdf).pvalue > 1e-3
    assert stats.kstest(phi[:, 1], stats.uniform(0, 1).cdf).pvalue > 1e-3
    assert np.allclose(lp, [O.prior_logpdf(cfg, p) for p in phi[:50]] + list(lp[50:]))


def test_rw_proposal_covariance():
    D = 3
    rw = np.array([[0.04, 0.01, 0.0], [0.01, 0.09, -0.02], [0.0, -0.02, 0.01]])
    cfg = _cfg(D, rw=rw)
    phi = np.zeros((40000, D))
    phi_new, lp_new = O.propose_rw(cfg, 5, 3, phi)
    C = np.cov(phi_new.T)
    assert np.allclose(C, rw, atol=4e-3)
    assert np.allclose(phi_new.mean(0), 0, atol=4e-3)
    # k selects a different stream
    phi_new2, _ = O.propose_rw(cfg, 5, 4, phi)
    assert not np.allclose(phi_new, phi_new2)


def _state(rng, N, D):
    return dict(phi=rng.normal(size=(N, D)), lp=rng.normal(size=N) - 3, ll=rng.normal(size=N) * 5 - 100,
                logw=rng.normal(size=N))


def test_forward_kernel_is_target_ratio():
    rng = np.random.default_rng(3)
    N, D = 300, 3
    cfg = _cfg(D, O.L_FORWARD)
    st0 = _state(rng, N, D)
    st = {k: v.copy() for k, v in st0.items()}
    phi_new, lp_new = O.propose_rw(cfg, 9, 2, st["phi"])
    ll_new = rng.normal(size=N) * 5 - 100
    status, logw_pre, anc, rec = O.outer_update(cfg, 2, 9, st, phi_new, lp_new, ll_new)
    assert status == 0
    want = (st0["logw"] + (lp_new + ll_new)) - (st0["lp"] + st0["ll"])
    assert np.array_equal(logw_pre, want)


@pytest.mark.parametrize("lkernel,N", [(O.L_GAUSS_OPT, 2), (O.L_GAUSS_OPT, 40), (O.L_FORWARD, 40)])
def test_fallback_kernel_keeps_the_learned_density(lkernel, N):
    """Eq. l_weights needs a backward kernel that is a normalised density in
    theta_{k-1}. When the Gaussian fit is not used (forward-kernel setting, or a fit
    rejected: at N = 2 the 2D-dimensional covariance has rank one; at N = 40 with one
    ancestor the previous population is a single point) the kernel is the random
    walk's Gaussian read backwards, N(phi_{k-1}; phi_k, Sigma_RW), and a learned
    proposal's log q stays in the weight. Dropping both (the target ratio alone, right
    only for a symmetric q) fails this."""
    rng = np.random.default_rng(40 + N + lkernel)
    D = 2
    rw = np.array([[0.05, 0.01], [0.01, 0.03]])
    cfg = _cfg(D, lkernel, rw=rw)
    st0 = _state(rng, N, D)
    if N > 2:
        st0["phi"][:] = st0["phi"][0]
    st = {k: v.copy() for k, v in st0.items()}
    phi_new = st0["phi"] + rng.normal(size=(N, D)) * 0.7 + 0.4   # not a random-walk draw
    lp_new = rng.normal(size=N) - 3
    ll_new = rng.normal(size=N) * 5 - 100
    logq = rng.normal(size=N) - 2.0
    status, logw_pre, anc, rec = O.outer_update(cfg, 3, 5, st, phi_new, lp_new, ll_new, logq=logq)
    assert status == 0
    assert rec[4] == (1 if lkernel == O.L_GAUSS_OPT else 0)
    for i in range(N):
        logL = stats.multivariate_normal(phi_new[i], rw).logpdf(st0["phi"][i])
        want = st0["logw"][i] + (lp_new[i] + ll_new[i]) - (st0["lp"][i] + st0["ll"][i]) + logL - logq[i]
        assert logw_pre[i] == pytest.approx(want, rel=1e-12, abs=1e-10)
    # the random walk's own density cancels the backward kernel exactly
    st = {k: v.copy() for k, v in st0.items()}
    phi_rw, lp_rw = O.propose_rw(cfg, 5, 3, st0["phi"])
    _, lw_rw, _, rec = O.outer_update(cfg, 3, 5, st, phi_rw, lp_rw, ll_new)
    assert np.array_equal(lw_rw, (st0["logw"] + (lp_rw + ll_new)) - (st0["lp"] + st0["ll"]))


def test_gauss_opt_weights_against_scipy_conditional():
    rng = np.random.default_rng(4)
    N, D = 500, 4
    rw = np.diag([0.04, 0.01, 0.09, 0.02])
    cfg = _cfg(D, O.L_GAUSS_OPT, rw=rw)
    st0 = _state(rng, N, D)
    st = {k: v.copy() for k, v in st0.items()}
    phi_new, lp_new = O.propose_rw(cfg, 11, 3, st["phi"])
    ll_new = rng.normal(size=N) * 5 - 100
    status, logw_pre, anc, rec = O.outer_update(cfg, 3, 11, st, phi_new, lp_new, ll_new)
    assert status == 0 and rec[4] == 0
    om = np.exp(st0["logw"] - st0["logw"].max())
    om /= om.sum()
    Z = np.hstack([st0["phi"], phi_new])
    mu = np.average(Z, axis=0, weights=om)
    S = np.cov(Z.T, aweights=om, bias=True)
    A = np.linalg.solve(S[D:, D:], S[D:, :D]).T
    Sc = S[:D, :D] - A @ S[D:, :D]
    for i in range(0, N, 41):
        logL = stats.multivariate_normal(mu[:D] + A @ (phi_new[i] - mu[D:]), Sc).logpdf(st0["phi"][i])
        logq = stats.multivariate_normal(st0["phi"][i], rw).logpdf(phi_new[i])
        want = st0["logw"][i] + (lp_new[i] + ll_new[i]) - (st0["lp"][i] + st0["ll"][i]) + logL - logq
        assert logw_pre[i] == pytest.approx(want, rel=1e-10, abs=1e-9)


def test_record_ess_estimates_and_resampling():
    rng = np.random.default_rng(5)
    N, D = 257, 2
    cfg = _cfg(D, O.L_FORWARD, prior=[[O.PRIOR_LOGNORMAL, 0.0, 1.0]] * D)
    st = _state(rng, N, D)
    phi_new = rng.normal(size=(N, D))
    lp_new = np.zeros(N)
    ll_new = rng.normal(size=N) * 3
    st["lp"][:] = 0
    st["ll"][:] = 0
    st["logw"][:] = 0
    status, logw_pre, anc, rec = O.outer_update(cfg, 2, 77, st, phi_new, lp_new, ll_new)
    w = np.exp(logw_pre - logw_pre.max())
    wn = w / w.sum()
    assert rec[1] == pytest.approx(1 / np.sum(wn**2), rel=1e-12)            # ESS = l_k
    assert rec[1] == pytest.approx(w.sum() ** 2 / np.sum(w**2), rel=1e-12)  # Eq. recycling_I
    th = np.exp(phi_new)
    assert rec[6:6 + D] == pytest.approx(wn @ th, rel=1e-12)
    cov = np.cov(th.T, aweights=wn, bias=True)
    assert rec[6 + D:6 + D + D * D] == pytest.approx(cov.ravel(), rel=1e-10)
    assert rec[6 + D + D * D:6 + 2 * D + D * D] == pytest.approx(wn @ phi_new, rel=1e-12, abs=1e-14)
    assert rec[-2] == 0 and rec[-1] == 0  # random-walk proposal, no learned score
    resampled = rec[1] < N / 2
    assert bool(rec[2]) == resampled
    if resampled:
        q = np.floor(np.exp(logw_pre - logw_pre.max()) * 2.0**32).astype(np.uint64)
        wd = O.philox([0, 0, 2 << 16, 5 << 24], [77, 0])
        x64 = int(wd[0]) | (int(wd[1]) << 32)
        want, _ = paper_systematic(q, x64)
        assert np.array_equal(anc, want)
        assert np.array_equal(st["phi"], phi_new[anc])
        assert np.all(st["logw"] == 0)
    else:
        assert np.array_equal(anc, np.arange(N))


def test_ess_closed_forms():
    N, D = 64, 2
    cfg = _cfg(D, O.L_FORWARD)
    rng = np.random.default_rng(6)
    phi_new = rng.normal(size=(N, D))
    for logw_pre_target, ess_want in [(np.zeros(N), N), (np.r_[0.0, np.full(N - 1, -np.inf)], 1.0)]:
        st = dict(phi=phi_new.copy(), lp=np.zeros(N), ll=np.zeros(N), logw=np.zeros(N))
        status, logw_pre, anc, rec = O.outer_update(cfg, 2, 1, st, phi_new, np.zeros(N), logw_pre_target)
        assert rec[1] == pytest.approx(ess_want, rel=1e-14)
    # scale invariance of l_k
    st = dict(phi=phi_new.copy(), lp=np.zeros(N), ll=np.zeros(N), logw=np.zeros(N))
    v = rng.normal(size=N)
    _, _, _, r1 = O.outer_update(cfg, 2, 1, {k: a.copy() for k, a in st.items()}, phi_new, np.zeros(N), v)
    _, _, _, r2 = O.outer_update(cfg, 2, 1, {k: a.copy() for k, a in st.items()}, phi_new, np.zeros(N), v + 123.0)
    assert r1[1] == pytest.approx(r2[1], rel=1e-12)


def test_all_dead_is_reported():
    N, D = 16, 2
    cfg = _cfg(D, O.L_FORWARD)
    st = dict(phi=np.zeros((N, D)), lp=np.zeros(N), ll=np.zeros(N), logw=np.zeros(N))
    status, *_ = O.outer_update(cfg, 2, 1, st, np.zeros((N, D)), np.zeros(N), np.full(N, -np.inf))
    assert status == -4


def test_recycling_constants():
    rng = np.random.default_rng(8)
    D, K = 3, 6
    RL = O.record_len(D)
    rec = np.zeros((K, RL))
    rec[:, 1] = rng.uniform(10, 500, K)
    means = rng.normal(size=(K, D))
    covs = np.array([_spd(rng, D) for _ in range(K)])
    rec[:, 6:6 + D] = means
    rec[:, 6 + D:6 + D + D * D] = covs.reshape(K, -1)
    mean, cov, c = O.recycle(rec, D)
    assert c.sum() == pytest.approx(1.0, rel=1e-15)
    assert c == pytest.approx(rec[:, 1] / rec[:, 1].sum(), rel=1e-15)
    assert mean == pytest.approx(c @ means, rel=1e-13)
    # mixture covariance: sum c_k (C_k + m_k m_k^T) - m m^T
    want = sum(c[k] * (covs[k] + np.outer(means[k], means[k])) for k in range(K)) - np.outer(mean, mean)
    assert np.allclose(cov, want, rtol=1e-12)
    rec[:, 1] = 42.0
    mean, _, c = O.recycle(rec, D)
    assert np.allclose(c, 1 / K) and mean == pytest.approx(means.mean(0), rel=1e-13)


def test_lkernel_fit_rejects_rounding_level_spread():
    """A population whose (phi_{k-1}) values coincide is degenerate even when the
    weighted sums leave rounding noise in the covariance; the fit must be rejected
    (not conditioned on that noise). So must a rank-deficient phi_{k-1} block."""
    rng = np.random.default_rng(3)
    N = 200
    phi = np.full((N, 2), [0.1234567, -2.71828])
    phi_new = phi + 0.3 * rng.normal(size=(N, 2))
    omega = rng.random(N)
    omega /= omega.sum()
    st, *_ = O.lkernel_fit(phi, phi_new, omega)
    assert st == -1
    x = rng.normal(size=N)
    phi = np.stack([x, 3.0 * x + 0.7], axis=1)
    st, *_ = O.lkernel_fit(phi, phi + 0.3 * rng.normal(size=(N, 2)), omega)
    assert st == -1


@pytest.mark.parametrize("spread", [1e-3, 1e-4])
def test_lkernel_fit_accepts_small_genuine_spread(spread):
    """A narrow but genuine population (relative spread far above the floor) is fitted."""
    rng = np.random.default_rng(4)
    N = 300
    phi = np.array([-11.5, 0.4]) + spread * rng.normal(size=(N, 2))
    phi_new = phi + spread * rng.normal(size=(N, 2))
    omega = np.full(N, 1.0 / N)
    st, mu, A, LS = O.lkernel_fit(phi, phi_new, omega)
    assert st == 0
    # conditional variance of phi_{k-1} given phi_k: half the marginal for equal variances
    assert np.allclose(np.diag(LS @ LS.T), 0.5 * spread**2, rtol=0.3)
