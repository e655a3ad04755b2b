"""Pins of the reference's learned Gaussian proposal (oracle/mlp.inc).

* Gradients of the plain FP64 network (bf16 off) against central finite differences,
  for every parameter block; the NLL gradient with respect to the outputs likewise.
* The NLL against scipy's multivariate normal with covariance L L^T.
* BF16 mode: when every matrix-product operand is already BF16-representable it
  equals the FP64 network exactly; round-to-nearest-even on known values.
* Adam: the first step moves every parameter by lr against the sign of its gradient.
* The random affine permutations are bijections for prime, even and odd N.
* Training on a Gaussian population (random pairing, uniform weights) learns the
  population's mean and covariance, and then beats the random walk on held-out pairs.
* The proposal density (with the Jacobian of the normalisation) against scipy.
* End to end: SMC^2 with the learned proposal still targets the exact grid posterior
  of the tiny SIR problem (a wrong density would bias it).
"""
import numpy as np
import pytest
from scipy import linalg, stats

import oracle as O
from paper_2311_12973_amd import workloads as W
from tests import exact_models as X


def _loss(D, w, rows, bf16=False):
    tot = 0.0
    for (u, ut, c) in rows:
        o, _, _ = O.mlp_forward(D, w, u, bf16=bf16)
        tot += c * O.mlp_nll(D, o, ut)
    return tot


def _grad(D, w, rows, bf16=False):
    g = np.zeros(O.mlp_nparams(D))
    for (u, ut, c) in rows:
        o, h1, h2 = O.mlp_forward(D, w, u, bf16=bf16)
        _, go = O.mlp_nll(D, o, ut, grad=True)
        g += O.mlp_backward(D, w, u, h1, h2, c * go, bf16=bf16)
    return g


@pytest.mark.parametrize("D", [2, 4, 5])
def test_gradients_match_finite_differences(D):
    rng = np.random.default_rng(D)
    w = O.mlp_init(D, 3).astype(np.float32)
    # move away from the initial point so every block (incl. off-diagonal L) matters
    w += (0.3 * rng.standard_normal(w.size)).astype(np.float32)
    rows = [(rng.normal(size=D), rng.normal(size=D) * 1.5, rng.uniform(0.5, 2.0)) for _ in range(3)]
    g = _grad(D, w, rows)
    H, P = O.MLP_H, O.mlp_nout(D)
    blocks = [0, H * D, H * D + H, H * D + H + H * H, H * D + 2 * H + H * H, H * D + 2 * H + H * H + P * H,
              O.mlp_nparams(D)]
    h = 2.0**-10
    for b in range(6):
        idx = rng.choice(np.arange(blocks[b], blocks[b + 1]), size=min(8, blocks[b + 1] - blocks[b]), replace=False)
        if b == 5:  # include the Cholesky diagonal and an off-diagonal output bias
            idx = np.unique(np.concatenate([idx, [blocks[5] + D, blocks[5] + D + 1]]))
        for i in idx:
            wp, wm = w.copy(), w.copy()
            wp[i] += np.float32(h)
            wm[i] -= np.float32(h)
            fd = (_loss(D, wp, rows) - _loss(D, wm, rows)) / (2 * h)
            assert fd == pytest.approx(g[i], rel=2e-4, abs=2e-6), (b, i)


@pytest.mark.parametrize("D", [1, 3, 8])
def test_nll_and_output_gradient(D):
    rng = np.random.default_rng(10 + D)
    P = O.mlp_nout(D)
    o = rng.normal(size=P)
    ut = rng.normal(size=D) * 2
    val, g = O.mlp_nll(D, o, ut, grad=True)
    L = np.zeros((D, D))
    for i in range(D):
        for j in range(i + 1):
            x = o[D + i * (i + 1) // 2 + j]
            L[i, j] = np.log1p(np.exp(x)) + 1e-3 if i == j else x
    ref = -stats.multivariate_normal(o[:D], L @ L.T).logpdf(ut)
    assert val == pytest.approx(ref, rel=1e-10)
    for p in range(P):
        op, om = o.copy(), o.copy()
        op[p] += 1e-6
        om[p] -= 1e-6
        fd = (O.mlp_nll(D, op, ut) - O.mlp_nll(D, om, ut)) / 2e-6
        assert fd == pytest.approx(g[p], rel=1e-5, abs=1e-7), p


def _bf16(x):
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def test_bf16_mode_is_exact_on_representable_operands():
    """With weights, inputs and hidden activations exactly representable in BF16 the
    rounding is the identity; tanh outputs are not, so a network whose hidden layers
    are saturated (|tanh| = 1 exactly in FP64) gives identical outputs in both modes."""
    D = 3
    H = O.MLP_H
    rng = np.random.default_rng(4)
    w = _bf16(O.mlp_init(D, 5) + 0.1 * rng.standard_normal(O.mlp_nparams(D)))  # BF16-representable
    sgn = np.where(np.arange(H) % 2 == 0, 32.0, -32.0).astype(np.float32)
    w[H * D:H * D + H] = sgn                      # b1 = +-32: every |tanh| is 1 in FP64
    w[H * D + H + H * H:H * D + 2 * H + H * H] = -sgn  # b2 likewise
    u = _bf16(np.array([1.5, -2.0, 0.75]))
    o1, h1, g1 = O.mlp_forward(D, w, u, bf16=True)
    o0, h0, g0 = O.mlp_forward(D, w, u, bf16=False)
    assert np.all(np.abs(h0) == 1.0) and np.all(np.abs(g0) == 1.0)
    assert np.array_equal(o1, o0)
    # and on generic inputs the two modes differ by BF16 rounding only
    o2, _, _ = O.mlp_forward(D, O.mlp_init(D, 6), np.array([0.3, -0.7, 1.1]), bf16=True)
    o3, _, _ = O.mlp_forward(D, O.mlp_init(D, 6), np.array([0.3, -0.7, 1.1]), bf16=False)
    assert np.allclose(o2, o3, rtol=2e-2, atol=1e-3) and not np.array_equal(o2, o3)
    # round to nearest even on known values
    assert _bf16(1.0 + 2.0**-8) == 1.0                    # tie -> even
    assert _bf16(1.0 + 3 * 2.0**-8) == 1.0 + 2.0**-6      # tie -> even (up)
    assert _bf16(1.0 + 2.0**-8 + 2.0**-12) == 1.0 + 2.0**-7


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(2)
    n = 50
    p = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n, dtype=np.float32)
    v = np.zeros(n, dtype=np.float32)
    g = rng.normal(size=n) * 10.0 ** rng.uniform(-3, 3, n)
    p0 = p.copy()
    O.adam_step(p, m, v, g, 1, 1e-3)
    assert np.allclose(p0 - p, 1e-3 * np.sign(g), rtol=1e-4, atol=1e-9)
    p1 = p.copy()
    O.adam_step(p, m, v, g, 2, 1e-3)  # constant gradient: still lr sign(g)
    assert np.allclose(p1 - p, 1e-3 * np.sign(g), rtol=1e-4, atol=1e-9)


@pytest.mark.parametrize("N", [2, 97, 256, 1000, 4096, 6561])
def test_permutations_are_bijections(N):
    for e in range(3):
        for which in range(2):
            a, b = O.mlp_perm(11, 3, e, which, N)
            img = (a * np.arange(N, dtype=np.uint64) + b) % N
            assert len(np.unique(img)) == N


def test_training_learns_a_gaussian_population():
    D = 3
    rng = np.random.default_rng(0)
    N = 1024
    mu = np.array([0.5, -1.0, 2.0])
    A = np.array([[0.3, 0, 0], [0.1, 0.2, 0], [-0.05, 0.1, 0.4]])
    phi = mu + rng.standard_normal((N, D)) @ A.T
    cfg = O.make_config(O.SEIR, O.OBS_NB_INC, D + 1, O.PREC_FP64, 1e6, [[O.PRIOR_NORMAL, 0, 5]] * (D + 1),
                        0.01 * np.eye(D + 1), [10.0], proposal=O.PROP_MLP, mlp_epochs=20, mlp_batch=128, mlp_lr=3e-3)
    cfg.D = D
    w = O.mlp_init(D, 1)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    t = 0
    for k in range(1, 4):
        use, t, frame, nm, nr = O.mlp_train(cfg, phi, np.zeros(N), 7, k, w, m, v, t)
    assert use == 1 and nm < nr
    # outputs at a few inputs: a Gaussian close to the population's
    c, F = frame[:D], frame[D:].reshape(D, D)
    for x in phi[:5]:
        o, _, _ = O.mlp_forward(D, w, linalg.solve_triangular(F, x - c, lower=True))
        L = np.zeros((D, D))
        for i in range(D):
            for j in range(i + 1):
                y = o[D + i * (i + 1) // 2 + j]
                L[i, j] = np.log1p(np.exp(y)) + 1e-3 if i == j else y
        mean = c + F @ o[:D]
        cov = F @ L @ L.T @ F.T
        assert np.allclose(mean, mu, atol=0.1)
        assert np.allclose(cov, A @ A.T, atol=0.04)


def _random_frame(rng, D):
    F = np.tril(rng.normal(scale=0.5, size=(D, D)), -1) + np.diag(rng.uniform(0.1, 3.0, D))
    return np.concatenate([rng.normal(size=D), F.ravel()])


def test_frame_is_the_weighted_gaussian_fit():
    """The frame holds the weighted mean and the lower Cholesky factor of the weighted
    covariance; a population with a constant coordinate falls back to the diagonal of
    standard deviations (floored at 1e-6)."""
    rng = np.random.default_rng(11)
    N, D = 500, 4
    phi = rng.normal(size=(N, D)) @ rng.normal(size=(D, D)) + rng.normal(size=D)
    wn = rng.uniform(0, 1, N)
    wn /= wn.sum()
    fr = O.mlp_frame(phi, wn)
    F = fr[D:].reshape(D, D)
    assert np.allclose(fr[:D], np.average(phi, axis=0, weights=wn), rtol=1e-12, atol=1e-12)
    assert np.array_equal(F, np.tril(F)) and np.all(np.diag(F) > 0)
    assert np.allclose(F @ F.T, np.cov(phi.T, aweights=wn, bias=True), rtol=1e-10, atol=1e-12)
    phi[:, 2] = 0.7
    fr = O.mlp_frame(phi, wn)
    sd = np.sqrt(np.maximum(np.diag(np.cov(phi.T, aweights=wn, bias=True)), 0))
    assert np.allclose(fr[D:].reshape(D, D), np.diag(np.maximum(sd, 1e-6)), rtol=1e-10, atol=1e-15)


def test_proposal_density_with_normalisation_jacobian():
    D = 4
    rng = np.random.default_rng(5)
    frame = _random_frame(rng, D)
    o = rng.normal(size=O.mlp_nout(D))
    L = np.zeros((D, D))
    for i in range(D):
        for j in range(i + 1):
            x = o[D + i * (i + 1) // 2 + j]
            L[i, j] = np.log1p(np.exp(x)) + 1e-3 if i == j else x
    F = frame[D:].reshape(D, D)
    dist = stats.multivariate_normal(frame[:D] + F @ o[:D], F @ L @ L.T @ F.T)
    draws = []
    for i in range(4000):
        phn, lq = O.mlp_propose_one(D, frame, o, 9, 3, i)
        if i < 20:
            assert lq == pytest.approx(dist.logpdf(phn), rel=1e-10, abs=1e-10)
        draws.append(phn)
    draws = np.array(draws)
    assert np.allclose(draws.mean(0), dist.mean, atol=4 * np.sqrt(np.diag(dist.cov) / 4000))
    assert np.allclose(np.cov(draws.T), dist.cov, rtol=0.1, atol=0.02)


N_POP, I0, T = 12, 2, 5
TRUTH = [0.85, 0.2]
MED, SD = (0.8, 0.2), 0.5


def _grid_posterior():
    """Exact posterior mean and standard deviation of (beta, gamma) for the tiny SIR
    problem on a grid of the log-normal prior's coordinates."""
    y = W.simulate(W.SIR, W.OBS_POIS_PREV, N_POP, TRUTH, T, seed=4, fixed=[I0], min_frac=0)
    G = 80
    pb = np.log(MED[0]) + SD * np.linspace(-5.5, 5.5, G)
    pg = np.log(MED[1]) + SD * np.linspace(-5.5, 5.5, G)
    ll = X.sir_grid_loglik(np.exp(pb), np.exp(pg), N_POP, I0, y, X.POIS_PREV)
    lpri = -0.5 * ((pb[:, None] - np.log(MED[0])) / SD) ** 2 - 0.5 * ((pg[None, :] - np.log(MED[1])) / SD) ** 2
    lw = ll + lpri
    wg = np.exp(lw - lw.max())
    wg /= wg.sum()
    B, Gm = np.exp(pb)[:, None], np.exp(pg)[None, :]
    mean = np.array([(wg * B).sum(), (wg * Gm).sum()])
    sd = np.sqrt([(wg * (B - mean[0]) ** 2).sum(), (wg * (Gm - mean[1]) ** 2).sum()])
    return y, mean, sd


@pytest.mark.slow
def test_learned_proposal_targets_the_grid_posterior():
    y, grid_mean, _ = _grid_posterior()
    prior = [[O.PRIOR_LOGNORMAL, np.log(MED[0]), SD], [O.PRIOR_LOGNORMAL, np.log(MED[1]), SD]]
    cfg = O.make_config(O.SIR, O.OBS_POIS_PREV, 2, O.PREC_FP64, N_POP, prior, 0.05 * np.eye(2), [I0],
                        proposal=O.PROP_MLP, mlp_epochs=4, mlp_batch=256, mlp_lr=3e-3)
    ests, used = [], 0
    for seed in range(1, 13):
        out = O.smc2_run(cfg, y, nx=48, seed=seed, N=2048, K=8)
        assert out["status"] == 0
        used += int(out["rec"][1:, -2].sum())
        mean, _, _ = O.recycle(out["rec"], 2)
        ests.append(mean)
    assert used > 0  # the learned proposal was actually used
    ests = np.array(ests)
    se = ests.std(0, ddof=1) / np.sqrt(len(ests))
    err = np.abs(ests.mean(0) - grid_mean)
    assert np.all(err < 4 * se + 2e-3), (ests.mean(0), grid_mean, se)


@pytest.mark.slow
def test_learned_proposal_with_the_forward_kernel_targets_the_grid_posterior():
    """With the forward-kernel setting every learned iteration is weighted through the
    fallback kernel N(phi_{k-1}; phi_k, Sigma_RW) and the network's exact density
    (Eq. l_weights). Weighting by the target ratio alone (valid only for a symmetric
    q) narrows the posterior to about half its width and moves its mean by ~5
    standard errors here; the pooled posterior spread and mean pin both terms."""
    y, grid_mean, grid_sd = _grid_posterior()
    prior = [[O.PRIOR_LOGNORMAL, np.log(MED[0]), SD], [O.PRIOR_LOGNORMAL, np.log(MED[1]), SD]]
    cfg = O.make_config(O.SIR, O.OBS_POIS_PREV, 2, O.PREC_FP64, N_POP, prior, 0.05 * np.eye(2), [I0],
                        lkernel=O.L_FORWARD, proposal=O.PROP_MLP, mlp_epochs=4, mlp_batch=256, mlp_lr=3e-3)
    ests, second, used = [], [], 0
    for seed in range(1, 13):
        out = O.smc2_run(cfg, y, nx=48, seed=seed, N=1024, K=8)
        assert out["status"] == 0
        used += int(out["rec"][1:, -2].sum())
        mean, cov, _ = O.recycle(out["rec"], 2)
        ests.append(mean)
        second.append(np.diag(cov) + mean ** 2)
    assert used >= 24  # the learned proposal drew most iterations
    ests = np.array(ests)
    se = ests.std(0, ddof=1) / np.sqrt(len(ests))
    assert np.all(np.abs(ests.mean(0) - grid_mean) < 4 * se + 2e-3), (ests.mean(0), grid_mean, se)
    pooled_sd = np.sqrt(np.mean(second, 0) - ests.mean(0) ** 2)
    assert np.all(np.abs(pooled_sd / grid_sd - 1) < 0.2), (pooled_sd, grid_sd)
