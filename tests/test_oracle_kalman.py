"""The reference particle filter against the Kalman filter on a scalar linear-Gaussian
model, where the log-likelihood has a closed form. The model shares with the epidemic
models every model-independent part of the filter (Sec. II): the weight recursion, the
likelihood increment with the mean-weight reset after resampling, the exact ESS trigger
and the integer systematic ancestors. A mistake in any of them (a dropped log S_prev,
no reset of the weights, a biased ancestor rule) biases the estimate of the likelihood,
which these tests see."""
import numpy as np
import pytest

import oracle as O

PHI, SQ, SR, M0, S0 = 0.9, 1.0, 1.0, 0.0, 1.0


def kalman_loglik(phi, sq, sr, m0, s0, y):
    """Exact log p(y_1:T) of x_0 ~ N(m0, s0^2), x_t = phi x_{t-1} + sq e_t,
    y_t = x_t + sr d_t (prediction-error decomposition)."""
    m, P, ll = m0, s0 * s0, 0.0
    for yt in y:
        m, P = phi * m, phi * phi * P + sq * sq
        S = P + sr * sr
        v = yt - m
        ll += -0.5 * (np.log(2.0 * np.pi * S) + v * v / S)
        K = P / S
        m, P = m + K * v, (1.0 - K) * P
    return ll


def simulate(T, seed):
    rng = np.random.default_rng(seed)
    x = M0 + S0 * rng.standard_normal()
    y = np.empty(T)
    for t in range(T):
        x = PHI * x + SQ * rng.standard_normal()
        y[t] = x + SR * rng.standard_normal()
    return y


def test_kalman_reference_on_a_hand_case():
    # one observation: y_1 ~ N(phi m0, phi^2 s0^2 + sq^2 + sr^2)
    ll = kalman_loglik(0.5, 2.0, 1.5, 1.0, 3.0, [0.7])
    var = 0.25 * 9.0 + 4.0 + 2.25
    assert ll == pytest.approx(-0.5 * (np.log(2 * np.pi * var) + (0.7 - 0.5) ** 2 / var), rel=1e-14)


def kalman_pin_statistic(pf_always=0, resampling=O.RS_SYSTEMATIC, M=2000):
    """Mean and standard error of exp(ll - ll_Kalman) over M independent filters."""
    y = simulate(25, 11)
    ref = kalman_loglik(PHI, SQ, SR, M0, S0, y)
    r = np.array([np.exp(O.pf_lg(PHI, SQ, SR, M0, S0, y, 64, 7, filt=f, pf_always=pf_always,
                                 resampling=resampling) - ref) for f in range(M)])
    return r.mean(), r.std(ddof=1) / np.sqrt(M)


@pytest.mark.parametrize("resampling", [O.RS_SYSTEMATIC, O.RS_MULTINOMIAL])
@pytest.mark.parametrize("pf_always", [0, 1])
def test_likelihood_estimate_is_unbiased(pf_always, resampling):
    mean, se = kalman_pin_statistic(pf_always, resampling)
    assert abs(mean - 1.0) < 4 * se + 1e-3, (mean, se)


def test_large_filter_converges_to_the_exact_likelihood():
    y = simulate(25, 12)
    ref = kalman_loglik(PHI, SQ, SR, M0, S0, y)
    est = np.array([O.pf_lg(PHI, SQ, SR, M0, S0, y, 40000, 3, filt=f) for f in range(4)])
    assert abs(est.mean() - ref) < 0.02, (est, ref)
    assert est.std() < 0.08


def test_increments_sum_to_the_estimate_and_resampling_is_adaptive():
    y = simulate(40, 13)
    ll, inc, rs = O.pf_lg(PHI, SQ, SR, M0, S0, y, 256, 5, trace=True)
    assert ll == pytest.approx(inc.sum(), rel=1e-12)
    assert rs[-1] == 0 and 0 < rs.sum() < len(y) - 1
    _, _, rs1 = O.pf_lg(PHI, SQ, SR, M0, S0, y, 256, 5, pf_always=1, trace=True)
    assert rs1[:-1].all() and rs1[-1] == 0


def test_deterministic_special_case_gives_the_exact_likelihood_and_states():
    # sq = s0 = 0: every particle follows x_t = phi^t m0 exactly, every weight is equal,
    # so the estimate is the exact likelihood and no day resamples
    phi, sr, m0 = 0.8, 0.7, 2.5
    y = simulate(12, 14)
    ll, inc, rs, xs = O.pf_lg(phi, 0.0, sr, m0, 0.0, y, 96, 9, trace=True, states=True, k=3)
    x, ref = m0, 0.0
    for t in range(len(y)):
        x = phi * x
        assert np.all(xs[t] == x), t
        ref += -0.5 * np.log(2 * np.pi * sr * sr) - 0.5 * ((y[t] - x) / sr) ** 2
    assert ll == pytest.approx(ref, rel=1e-13)
    assert not rs.any()


def test_iteration_index_selects_independent_streams():
    y = simulate(20, 15)
    a = O.pf_lg(PHI, SQ, SR, M0, S0, y, 64, 7, filt=3, k=0)
    b = O.pf_lg(PHI, SQ, SR, M0, S0, y, 64, 7, filt=3, k=1)
    c = O.pf_lg(PHI, SQ, SR, M0, S0, y, 64, 7, filt=3, k=1)
    assert a != b and b == c
    # the estimate stays unbiased on the streams of a later iteration
    ref = kalman_loglik(PHI, SQ, SR, M0, S0, simulate(25, 11))
    r = np.array([np.exp(O.pf_lg(PHI, SQ, SR, M0, S0, simulate(25, 11), 64, 7, filt=f, k=5) - ref)
                  for f in range(2000)])
    assert abs(r.mean() - 1.0) < 4 * r.std(ddof=1) / np.sqrt(len(r)) + 1e-3


def test_kalman_recursion_equals_the_joint_gaussian():
    # the prediction-error decomposition against the joint density of y_1:T written out
    from tests.exact_models import kalman_loglik_grid, lingauss_loglik_joint
    y = simulate(7, 16)
    for (a, sx, sy, m0, s0) in [(0.9, 1.0, 1.0, 0.0, 1.0), (-0.6, 0.4, 1.7, 1.5, 0.3), (1.1, 2.0, 0.5, -1.0, 0.0)]:
        ref = lingauss_loglik_joint(a, sx, sy, m0, s0, y)
        assert kalman_loglik(a, sx, sy, m0, s0, y) == pytest.approx(ref, rel=1e-12)
        assert kalman_loglik_grid(np.array([a, a]), sx, sy, m0, s0, y) == pytest.approx([ref, ref], rel=1e-12)


def test_iteration_index_reaches_the_resampling_stream():
    # no state noise: the states of day 2 are PHI times the day-1 states picked by the
    # day-1 ancestors, which must come from the uniforms of counter word k<<16 | 1
    y = simulate(3, 17)
    for k in (0, 1, 5):
        _, _, rs, xs = O.pf_lg(PHI, 0.0, SR, M0, S0, y, 64, 7, filt=2, pf_always=1, trace=True, k=k, states=True,
                               resampling=O.RS_MULTINOMIAL)
        assert rs[0] == 1
        a = -0.5 * ((y[0] - xs[0]) / SR) ** 2
        w = np.exp(a - a.max())
        q = np.where(w >= 1.0, 2 ** 32, np.floor(w * 2.0 ** 32)).astype(np.uint64)
        anc = O.resample_multinomial(q, 7, 2, (k << 16) | 1)
        assert np.array_equal(xs[1], PHI * xs[0][anc]), k
