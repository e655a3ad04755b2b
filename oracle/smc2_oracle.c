/*
 * smc2_oracle.c — plain, slow CPU reference of the SMC^2 sampler of Rosato, Varsi,
 * Murphy and Maskell (arXiv 2311.12973). TEST INFRASTRUCTURE ONLY: the tests, the
 * smoke check and the CPU-baseline leg of the benchmark are its only users; the
 * product path never loads it. It shares no code with the GPU library.
 *
 * Conventions both implementations follow (the paper leaves them open):
 *
 *  Random numbers. Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 *  numbers: as easy as 1, 2, 3", SC'11), key = (seed low word, seed high word),
 *  counter (c0, c1, c2, c3):
 *    particle-filter flows : (j particle, i filter, k<<16 | t, 1<<24 | b<<16 | call)
 *    particle-filter resampling : (0, i, k<<16 | t, 2<<24)
 *    prior draw           : (i sample, 0, 1<<16, 3<<24 | d)
 *    random-walk normal   : (i sample, 0, k<<16, 4<<24 | d)
 *    outer resampling     : (0, 0, k<<16, 5<<24)
 *  Uniforms: u24(x) = (2*(x>>9)+1) * 2^-24 (exact in FP32), u53(lo,hi) =
 *  (2*((hi:lo)>>12)+1) * 2^-53. Normals: Box-Muller on (u53(w0,w1), u53(w2,w3)),
 *  first output only.
 *
 *  Integer systematic resampling (Sec. IV-B, Eq. cdf / ncopies, used for the
 *  particle filter too): q_j = floor(2^32 * exp(a_j - max a)), C_j = sum_{l<=j} q_l,
 *  Q = C_{n-1}, U = floor(x64 * Q / 2^64) with x64 a 64-bit Philox output, and
 *  ancestor(m) = min{ j : n*C_j > m*Q + U }. This is the paper's ceil form with
 *  cdf_j = n*C_j/Q and u = U/Q in [0,1): ncopies_j = #{m : n*C_{j-1} <= m*Q+U < n*C_j}
 *  (a point on a boundary goes to the upper index).
 *  Trigger ESS < n/2 evaluated exactly on q'_j = q_j >> 8: 2*(sum q')^2 < n*sum q'^2.
 *
 *  L-kernel (Sec. IV-D): Gaussian fitted to the pairs (phi_{k-1}^i, phi_k^i) with the
 *  normalised weights of iteration k-1, then conditioned (textbook Gaussian
 *  conditioning): L = N(phi_{k-1}; mu_1 + A (phi_k - mu_2), S), A = S12 S22^-1,
 *  S = S11 - A S21. The forward-kernel setting, and a rejected fit, use the random
 *  walk's Gaussian read backwards, L = N(phi_{k-1}; phi_k, Sigma_RW): for the random
 *  walk this is the paper's forward kernel (the weight becomes the target ratio), and
 *  for a learned proposal it is still a normalised density in phi_{k-1}, so the
 *  proposal's own density stays in the weight.
 *
 *  Parameters live on sampler coordinates phi (identity for a uniform prior, log for
 *  a log-normal prior, logit for a logit-normal prior); the proposal, the L-kernel
 *  and the prior density are all on phi; the model sees theta(phi).
 */
#include "smc2_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LOG_2PI 1.8378770664093453

int or_record_len(int D) { return 8 + 2 * D + D * D; }
int or_n_obs(int model) { return model == OR_AGE_SEIR ? 4 : 1; }

/* ------------------------------------------------------------------ random numbers */

void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

float or_u24(uint32_t x) { return (float)((double)(2u * (x >> 9) + 1u) * 0x1p-24); }

double or_u53(uint32_t lo, uint32_t hi)
{
    uint64_t x = ((uint64_t)hi << 32) | lo;
    return (double)(2u * (x >> 12) + 1u) * 0x1p-53;
}

double or_normal_call(uint64_t seed, const uint32_t ctr[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    or_philox(ctr, key, w);
    double u1 = or_u53(w[0], w[1]);
    double u2 = or_u53(w[2], w[3]);
    double rad = sqrt(-2.0 * log(u1));
    return rad * cos(6.283185307179586 * u2);
}

/* ------------------------------------------------------------------ observations */

/* The observation log-pmf (Sec. V-A: Poisson; the negative binomial has mean `count`
 * and dispersion r) split into a per-day constant that does not depend on the
 * particle and a per-particle part, both in FP64:
 *   Poisson:  log g = [y log(lambda) - lambda]                          + [-lgamma(y+1)]
 *   NB:       log g = -[y log1p(r/mu) + r log1p(mu/r)]
 *                     + [lgamma(y+r) - lgamma(r) - lgamma(y+1)]
 * The per-particle parts have no cancellation (the NB part is a sum of two
 * non-negative terms), so their rounding to the filter precision is well defined.
 * A zero mean gives 0 for y = 0 and -inf otherwise. */
static double or_obs_const(int obs, int32_t y, double r)
{
    if (obs == OR_OBS_NB_INC) return (lgamma((double)y + r) - lgamma(r)) - lgamma((double)y + 1.0);
    return -lgamma((double)y + 1.0);
}

static double or_obs_part(int obs, int32_t y, int32_t cnt, double r)
{
    if (cnt <= 0) return (y == 0) ? 0.0 : -INFINITY;
    const double mu = (double)cnt;
    if (obs == OR_OBS_NB_INC) return -((double)y * log1p(r / mu) + r * log1p(mu / r));
    return (double)y * log(mu) - mu;
}

double or_obs_logpmf(int obs, int32_t y, int32_t count, double r)
{
    return or_obs_part(obs, y, count, r) + or_obs_const(obs, y, r);
}

/* ------------------------------------------------------------------ resampling */

int or_resample_trigger(const uint64_t* q, int n)
{
    /* q >> 8 <= 2^24, so for n < 2^31: s1 < 2^55, 2 s1^2 < 2^111 and n s2 < 2^110 -- exact in 128 bits */
    unsigned __int128 s1 = 0, s2 = 0;
    for (int j = 0; j < n; ++j) {
        const uint64_t v = q[j] >> 8;
        s1 += v;
        s2 += (unsigned __int128)v * v;
    }
    return s1 * s1 * 2u < s2 * (unsigned)n;
}

/* Systematic resampling (Eq. ncopies: ncopies^i = ceil(cdf^i - u) - ceil(cdf^{i-1} - u),
 * i.e. sample i receives the points m + u lying in [cdf^{i-1}, cdf^i)), then sequential
 * redistribution (Alg. 1). In integers: cdf^i = n*C_i/Q, u = U/Q, and the sorted points
 * m*Q + U are walked against the scaled cumulative sums n*C_j. */
void or_resample_ancestors(const uint64_t* q, int n, uint64_t x64, int32_t* anc)
{
    uint64_t* C = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t acc = 0;
    for (int j = 0; j < n; ++j) {
        acc += q[j];
        C[j] = acc;
    }
    uint64_t Q = acc;
    uint64_t U = (uint64_t)(((unsigned __int128)x64 * Q) >> 64);
    int j = 0;
    for (int m = 0; m < n; ++m) {
        const unsigned __int128 target = (unsigned __int128)m * Q + U;
        while ((unsigned __int128)n * C[j] <= target) ++j;
        anc[m] = j;
    }
    free(C);
}

/* ------------------------------------------------------------------ linear algebra */

/* Unpivoted lower Cholesky of the n x n matrix A (lower triangle read). Returns 0 on
 * success, -1 if a pivot is not strictly positive. */
int or_cholesky(int n, const double* A, double* L)
{
    memset(L, 0, sizeof(double) * (size_t)n * n);
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) return -1;
        L[j * n + j] = sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = v / L[j * n + j];
        }
    }
    return 0;
}

/* log N(x; mu, L L^T). */
double or_mvn_logpdf_chol(int n, const double* x, const double* mu, const double* L)
{
    double v[2 * OR_DMAX];
    double quad = 0.0, logdet = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = x[i] - mu[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * v[k];
        v[i] = s / L[i * n + i];
        quad += v[i] * v[i];
        logdet += log(L[i * n + i]);
    }
    return -0.5 * quad - logdet - 0.5 * n * LOG_2PI;
}

/* Solve (L L^T) x = b in place. */
static void chol_solve(int n, const double* L, double* b)
{
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
        b[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
        b[i] = s / L[i * n + i];
    }
}

/*
 * Approximately optimal L-kernel (Sec. IV-D, Eq. Gauss_joint and the conditional that
 * follows it, read as textbook Gaussian conditioning). Fits mean mu (2D) and
 * covariance (2D x 2D) of z_i = (phi_i, phi_new_i) with weights omega (summing to 1),
 * then returns A = S12 S22^{-1} and the Cholesky factor LS of S = S11 - A S21.
 * Returns 0, or -1 when a Cholesky factorisation fails.
 */
int or_lkernel_fit(int N, int D, const double* phi, const double* phi_new, const double* omega,
                   double* mu, double* A, double* LS)
{
    return or_lkernel_fit_cov(N, D, phi, phi_new, omega, mu, A, LS, NULL);
}

int or_lkernel_fit_cov(int N, int D, const double* phi, const double* phi_new, const double* omega,
                       double* mu, double* A, double* LS, double* cov_out)
{
    const int D2 = 2 * D;
    double cov[4 * OR_DMAX * OR_DMAX];
    for (int a = 0; a < D2; ++a) mu[a] = 0.0;
    for (int i = 0; i < N; ++i)
        for (int a = 0; a < D2; ++a) {
            double z = a < D ? phi[i * D + a] : phi_new[i * D + a - D];
            mu[a] += omega[i] * z;
        }
    for (int a = 0; a < D2 * D2; ++a) cov[a] = 0.0;
    for (int i = 0; i < N; ++i) {
        double z[2 * OR_DMAX];
        for (int a = 0; a < D2; ++a) z[a] = (a < D ? phi[i * D + a] : phi_new[i * D + a - D]) - mu[a];
        for (int a = 0; a < D2; ++a)
            for (int c = 0; c < D2; ++c) cov[a * D2 + c] += omega[i] * z[a] * z[c];
    }
    if (cov_out)
        for (int a = 0; a < D2 * D2; ++a) cov_out[a] = cov[a];
    /* Numerical-rank floor: a Cholesky pivot of coordinate a must exceed
       OR_LK_REL_FLOOR times that coordinate's raw second moment cov_aa + mu_a^2 (the
       scale of the rounding error of a variance computed from the samples); a fit
       of a (numerically) degenerate population is rejected instead of being
       conditioned on rounding noise. */
    double floor_[2 * OR_DMAX];
    for (int a = 0; a < D2; ++a) floor_[a] = OR_LK_REL_FLOOR * (cov[a * D2 + a] + mu[a] * mu[a]);
    double S22[OR_DMAX * OR_DMAX] = {0}, L22[OR_DMAX * OR_DMAX], S[OR_DMAX * OR_DMAX] = {0};
    for (int a = 0; a < D; ++a)
        for (int c = 0; c < D; ++c) S22[a * D + c] = cov[(D + a) * D2 + D + c];
    if (or_cholesky(D, S22, L22) != 0) return -1;
    for (int a = 0; a < D; ++a)
        if (!(L22[a * D + a] * L22[a * D + a] > floor_[D + a])) return -1;
    /* row r of A solves S22 a = S21[:, r] (S22 symmetric) */
    for (int r = 0; r < D; ++r) {
        double b[OR_DMAX];
        for (int c = 0; c < D; ++c) b[c] = cov[(D + c) * D2 + r];
        chol_solve(D, L22, b);
        for (int c = 0; c < D; ++c) A[r * D + c] = b[c];
    }
    for (int a = 0; a < D; ++a)
        for (int c = 0; c < D; ++c) {
            double s = cov[a * D2 + c];
            for (int e = 0; e < D; ++e) s -= A[a * D + e] * cov[(D + e) * D2 + c];
            S[a * D + c] = s;
        }
    if (or_cholesky(D, S, LS) != 0) return -1;
    for (int a = 0; a < D; ++a)
        if (!(LS[a * D + a] * LS[a * D + a] > floor_[a])) return -1;
    return 0;
}

/* ------------------------------------------------------------------ prior */

double or_prior_logpdf(const or_config* cfg, const double* phi)
{
    double lp = 0.0;
    for (int d = 0; d < cfg->D; ++d) {
        int fam = (int)cfg->prior[d][0];
        double a = cfg->prior[d][1], b = cfg->prior[d][2];
        if (fam == OR_PRIOR_UNIFORM) {
            if (!(phi[d] >= a && phi[d] <= b)) return -INFINITY;
            lp += -log(b - a);
        } else {
            double z = (phi[d] - a) / b;
            lp += (-0.5 * z * z - log(b)) - 0.5 * LOG_2PI;
        }
    }
    return lp;
}

void or_theta_of_phi(const or_config* cfg, const double* phi, double* theta)
{
    for (int d = 0; d < cfg->D; ++d) {
        int fam = (int)cfg->prior[d][0];
        if (fam == OR_PRIOR_LOGNORMAL) theta[d] = exp(phi[d]);
        else if (fam == OR_PRIOR_LOGITNORMAL) theta[d] = 1.0 / (1.0 + exp(-phi[d]));
        else theta[d] = phi[d];
    }
}

/* k = 1 importance sampling from q_1 = prior (Sec. IV-A, Eq. init_sample). */
void or_prior_draw(const or_config* cfg, int N, uint64_t seed, double* phi, double* lp)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int i = 0; i < N; ++i) {
        for (int d = 0; d < cfg->D; ++d) {
            uint32_t ctr[4] = {(uint32_t)i, 0u, 1u << 16, ((uint32_t)OR_S_PRIOR << 24) | (uint32_t)d};
            uint32_t w[4];
            or_philox(ctr, key, w);
            double u1 = or_u53(w[0], w[1]), u2 = or_u53(w[2], w[3]);
            int fam = (int)cfg->prior[d][0];
            double a = cfg->prior[d][1], b = cfg->prior[d][2];
            if (fam == OR_PRIOR_UNIFORM) {
                phi[i * cfg->D + d] = a + (b - a) * u1;
            } else {
                double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
                phi[i * cfg->D + d] = a + b * z;
            }
        }
        lp[i] = or_prior_logpdf(cfg, phi + (size_t)i * cfg->D);
    }
}

/* k > 1 Gaussian random-walk proposal (Sec. IV-A, Eq. proposal): phi' = phi + L z. */
void or_propose_rw(const or_config* cfg, int N, uint64_t seed, uint32_t k, const double* phi,
                   double* phi_new, double* lp_new)
{
    const int D = cfg->D;
    double C[OR_DMAX * OR_DMAX], L[OR_DMAX * OR_DMAX];
    for (int a = 0; a < D; ++a)
        for (int c = 0; c < D; ++c) C[a * D + c] = cfg->rw_cov[a][c];
    or_cholesky(D, C, L);
    for (int i = 0; i < N; ++i) {
        double z[OR_DMAX];
        for (int d = 0; d < D; ++d) {
            uint32_t ctr[4] = {(uint32_t)i, 0u, k << 16, ((uint32_t)OR_S_RW << 24) | (uint32_t)d};
            z[d] = or_normal_call(seed, ctr);
        }
        for (int d = 0; d < D; ++d) {
            double acc = 0.0;
            for (int e = 0; e <= d; ++e) acc += L[d * D + e] * z[e];
            phi_new[i * D + d] = phi[i * D + d] + acc;
        }
        lp_new[i] = or_prior_logpdf(cfg, phi_new + (size_t)i * D);
    }
}

/* Truncated Langevin proposal (a gradient-informed random walk; the drift shrunk to a
 * bounded length as in Roberts and Tweedie's truncated form). The gradient is the
 * particle filter's score estimate of the sample, which travelled with it like its
 * likelihood estimate, mapped to the sampler coordinates, plus the prior's gradient; the
 * proposal is then an exactly computable density given the sample's stored state. */
double or_propose_langevin_one(const or_config* cfg, const double* L, const double* phi, const double* s_theta,
                               uint64_t seed, uint32_t k, int i, double* phi_new)
{
    const int D = cfg->D;
    double th[OR_DMAX], g[OR_DMAX], v[OR_DMAX], delta[OR_DMAX], z[OR_DMAX], m[OR_DMAX];
    or_theta_of_phi(cfg, phi, th);
    for (int d = 0; d < D; ++d) {
        const int fam = (int)cfg->prior[d][0];
        const double a = cfg->prior[d][1], b = cfg->prior[d][2];
        const double J = fam == OR_PRIOR_LOGNORMAL ? th[d] : (fam == OR_PRIOR_LOGITNORMAL ? th[d] * (1.0 - th[d]) : 1.0);
        const double gp = fam == OR_PRIOR_UNIFORM ? 0.0 : -(phi[d] - a) / (b * b);
        g[d] = J * s_theta[d] + gp;
    }
    /* delta = 1/2 Sigma g = 1/2 L v with v = L' g; its Mahalanobis length |L^-1 delta| is |v| / 2 */
    double n2 = 0.0;
    for (int a = 0; a < D; ++a) {
        double acc = 0.0;
        for (int c = a; c < D; ++c) acc += L[c * D + a] * g[c];
        v[a] = acc;
        n2 += acc * acc;
    }
    const double len = 0.5 * sqrt(n2);
    const double shrink = len > 1.0 ? 1.0 / len : 1.0;
    const double step = cfg->lgv_step > 0.0 ? cfg->lgv_step : 0.25;
    for (int a = 0; a < D; ++a) {
        double acc = 0.0;
        for (int c = 0; c <= a; ++c) acc += L[a * D + c] * v[c];
        delta[a] = step * ((0.5 * acc) * shrink);
    }
    for (int d = 0; d < D; ++d) {
        uint32_t ctr[4] = {(uint32_t)i, 0u, k << 16, ((uint32_t)OR_S_RW << 24) | (uint32_t)d};
        z[d] = or_normal_call(seed, ctr);
    }
    for (int a = 0; a < D; ++a) {
        m[a] = phi[a] + delta[a];
        double acc = 0.0;
        for (int c = 0; c <= a; ++c) acc += L[a * D + c] * z[c];
        phi_new[a] = m[a] + acc;
    }
    return or_mvn_logpdf_chol(D, phi_new, m, L);
}

/* Multinomial resampling, the particle filter's scheme in Sec. II: every slot draws its
 * ancestor independently with probability q_j / Q, from its own 64-bit uniform
 * U_m = floor(x64_m Q / 2^64) and the first j with C_j > U_m (exact integers). */
void or_resample_multinomial(const uint64_t* q, int n, uint64_t seed, uint32_t filt, uint32_t kt, int32_t* anc)
{
    uint64_t* C = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t acc = 0;
    for (int j = 0; j < n; ++j) {
        acc += q[j];
        C[j] = acc;
    }
    const uint64_t Q = acc;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int m = 0; m < n; ++m) {
        const uint32_t ctr[4] = {(uint32_t)(m >> 1), filt, kt, ((uint32_t)OR_S_PF_RS << 24) | (1u << 16)};
        uint32_t w[4];
        or_philox(ctr, key, w);
        const uint64_t x64 = (m & 1) ? ((uint64_t)w[2] | ((uint64_t)w[3] << 32)) : ((uint64_t)w[0] | ((uint64_t)w[1] << 32));
        const uint64_t U = (uint64_t)(((unsigned __int128)x64 * Q) >> 64);
        int lo = 0, hi = n - 1; /* first j with C_j > U (exists: U < Q = C_{n-1}) */
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (C[mid] > U) hi = mid;
            else lo = mid + 1;
        }
        anc[m] = lo;
    }
    free(C);
}

/* ------------------------------------------------------------------ event counts
 * How often the particle filter performs each primitive of the method (particle-step,
 * binomial draw, inversion step, BTRS set-up, attempt and final test, Philox call,
 * FP64 transcendental, particle resampled). They feed the algorithmic operation count
 * per particle-step (the roofline's unit of work); counting changes no result. Each
 * thread counts in its own slots and adds them to the totals once per filter. */
static _Thread_local double tl_ev[OR_EV_N];
static double g_ev[OR_EV_N];
#define OR_EV(i, v) (tl_ev[(i)] += (v))

static void or_events_flush(void)
{
#pragma omp critical(or_events)
    for (int e = 0; e < OR_EV_N; ++e) {
        g_ev[e] += tl_ev[e];
        tl_ev[e] = 0.0;
    }
}

void or_events_get(double* out)
{
    for (int e = 0; e < OR_EV_N; ++e) out[e] = g_ev[e];
}

void or_events_reset(void)
{
    for (int e = 0; e < OR_EV_N; ++e) g_ev[e] = 0.0;
}

/* ------------------------------------------------------------------ particle filters */

/* The deterministic initial state x_0 of every particle (Sec. V-A: the initially
 * infected, the rest susceptible; SEIR models start with I_0 = round(iota N), at least
 * one and at most N, per group for the age-structured model, whose group sizes are
 * round(fraction N_pop)) and the negative-binomial dispersion r (0 where unused). */
static double or_model_start(const or_config* cfg, const double* th, int32_t* x0)
{
    if (cfg->model == OR_SIR) {
        int32_t i0 = (int32_t)cfg->fixed[0];
        x0[0] = (int32_t)cfg->n_pop - i0;
        x0[1] = i0;
        return 0.0;
    }
    if (cfg->model == OR_SEIR) {
        double i0 = floor(th[3] * cfg->n_pop + 0.5);
        if (i0 < 1.0) i0 = 1.0;
        if (i0 > cfg->n_pop) i0 = cfg->n_pop;
        x0[0] = (int32_t)(cfg->n_pop - i0);
        x0[1] = 0;
        x0[2] = (int32_t)i0;
        return (cfg->D >= 5) ? th[4] : cfg->fixed[0];
    }
    for (int g = 0; g < 4; ++g) {
        double ng = floor(cfg->fixed[16 + g] * cfg->n_pop + 0.5);
        double i0 = floor(th[3] * ng + 0.5);
        if (i0 < 1.0) i0 = 1.0;
        if (i0 > ng) i0 = ng;
        x0[3 * g] = (int32_t)(ng - i0);
        x0[3 * g + 1] = 0;
        x0[3 * g + 2] = (int32_t)i0;
    }
    return th[4];
}

/* Digamma psi(x) for x > 0 (FP64): the recurrence psi(x) = psi(x + 1) - 1/x up to
 * x >= 10, then the asymptotic series ln x - 1/(2x) - sum_k B_2k / (2k x^2k) with the
 * Bernoulli numbers B_2 .. B_14 (remainder below 1e-17 at x = 10). */
double or_digamma(double x)
{
    double acc = 0.0;
    while (x < 10.0) {
        acc = acc - 1.0 / x;
        x = x + 1.0;
    }
    const double r = 1.0 / x, r2 = r * r;
    const double series =
        r2 * (1.0 / 12 - r2 * (1.0 / 120 - r2 * (1.0 / 252 - r2 * (1.0 / 240 - r2 * (1.0 / 132 - r2 * (691.0 / 32760 - r2 * (1.0 / 12)))))));
    return acc + ((log(x) - 0.5 * r) - series);
}

#define REAL float
#define FN(x) x##_f32
#include "pf_real.inc"
#undef REAL
#undef FN
#define REAL double
#define FN(x) x##_f64
#include "pf_real.inc"
#undef REAL
#undef FN

int32_t or_binomial(int prec, int32_t n, double p, uint64_t seed, uint32_t j, uint32_t i,
                    uint32_t k, uint32_t t, uint32_t b)
{
    uint32_t kt = (k << 16) | t;
    if (prec == OR_PREC_FP32) return binom_f32(n, (float)p, seed, j, i, kt, b);
    return binom_f64(n, p, seed, j, i, kt, b);
}

/* count draws at particle coordinates j = 0..count-1 (same filter, iteration, day, draw). */
void or_binomial_batch(int prec, int32_t n, double p, uint64_t seed, uint32_t i, uint32_t k,
                       uint32_t t, uint32_t b, int count, int32_t* out)
{
    for (int j = 0; j < count; ++j) out[j] = or_binomial(prec, n, p, seed, (uint32_t)j, i, k, t, b);
}

/* count draws with per-draw (n[j], p[j]) at particle coordinates j = 0..count-1. */
void or_binomial_many(int prec, int count, const int32_t* n, const double* p, uint64_t seed, uint32_t i,
                      uint32_t k, uint32_t t, uint32_t b, int32_t* out)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < count; ++j) out[j] = or_binomial(prec, n[j], p[j], seed, (uint32_t)j, i, k, t, b);
}

/*
 * The same particle filter on a scalar linear-Gaussian state-space model, whose exact
 * log-likelihood the Kalman filter gives in closed form (a pin of the filter's weight
 * recursion, likelihood increments, mean-weight reset, trigger and ancestors, which
 * this model shares with the epidemic models through weigh_f64):
 *   x_0 ~ N(m0, s0^2),  x_t = phi x_{t-1} + sq e_t,  y_t = x_t + sr d_t,  e, d ~ N(0, 1).
 * Bootstrap proposal; normals from Box-Muller on the Philox counter
 * (particle j, filter, k<<16 | t, 8<<24) -- t = 0 draws x_0; the resampling uniforms
 * come from the epidemic filters' streams with the same k<<16 | t, so k selects the
 * iteration's streams throughout. FP64 throughout. x_out (T x nx, optional): the
 * states of each day before resampling.
 */
double or_pf_lg(double phi, double sq, double sr, double m0, double s0, const double* y, int T, int nx,
                uint64_t seed, uint32_t filt, uint32_t k, int pf_always, int resampling, double* inc_out,
                int32_t* rs_out, double* x_out, double* score_out)
{
    double* x = (double*)malloc(sizeof(double) * (size_t)nx);
    double* xs = (double*)malloc(sizeof(double) * (size_t)nx);
    double* lw = (double*)malloc(sizeof(double) * (size_t)nx);
    double* a = (double*)malloc(sizeof(double) * (size_t)nx);
    double* w = (double*)malloc(sizeof(double) * (size_t)nx);
    uint64_t* qq = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nx);
    int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)nx);
    /* score: running complete-data score of (phi, sq, sr) per particle; with the drawn
     * noise e = (x_t - phi x_{t-1}) / sq: d/dphi = e x_{t-1} / sq, d/dsq = (e^2 - 1) / sq,
     * and from the observation d/dsr = (z^2 - 1) / sr */
    double* sj = score_out ? (double*)calloc((size_t)nx * 3, sizeof(double)) : NULL;
    double* sjs = score_out ? (double*)malloc(sizeof(double) * (size_t)nx * 3) : NULL;
    for (int j = 0; j < nx; ++j) {
        uint32_t ctr[4] = {(uint32_t)j, filt, k << 16, 8u << 24};
        x[j] = m0 + s0 * or_normal_call(seed, ctr);
        lw[j] = 0.0;
    }
    double s_prev = (double)nx, ll = 0.0;
    const double cst = -log(sr) - 0.5 * log(2.0 * M_PI);
    for (int t = 1; t <= T; ++t) {
        for (int j = 0; j < nx; ++j) {
            uint32_t ctr[4] = {(uint32_t)j, filt, (k << 16) | (uint32_t)t, 8u << 24};
            const double e = or_normal_call(seed, ctr);
            const double xp = x[j];
            x[j] = phi * xp + sq * e;
            const double z = (y[t - 1] - x[j]) / sr;
            a[j] = lw[j] + -0.5 * z * z;
            if (sj) {
                double* sc = sj + (size_t)j * 3;
                sc[0] = sc[0] + (e * xp) / sq;
                sc[1] = sc[1] + (e * e - 1.0) / sq;
                sc[2] = sc[2] + (z * z - 1.0) / sr;
            }
        }
        if (x_out) memcpy(x_out + (size_t)(t - 1) * nx, x, sizeof(double) * (size_t)nx);
        double inc;
        const int rs = weigh_f64(nx, a, lw, w, qq, anc, &s_prev, cst, t < T, pf_always, resampling, seed, filt,
                                 (k << 16) | (uint32_t)t, &inc);
        if (inc_out) inc_out[t - 1] = inc;
        if (rs_out) rs_out[t - 1] = rs > 0;
        if (rs < 0) {
            ll = -INFINITY;
            break;
        }
        ll = ll + inc;
        if (rs) {
            for (int j = 0; j < nx; ++j) xs[j] = x[anc[j]];
            memcpy(x, xs, sizeof(double) * (size_t)nx);
            if (sj) {
                for (int j = 0; j < nx; ++j)
                    for (int d = 0; d < 3; ++d) sjs[(size_t)j * 3 + d] = sj[(size_t)anc[j] * 3 + d];
                memcpy(sj, sjs, sizeof(double) * (size_t)nx * 3);
            }
        }
    }
    if (score_out) { /* the final weights average the particles' scores */
        for (int d = 0; d < 3; ++d) score_out[d] = 0.0;
        if (ll != -INFINITY) {
            double S = 0.0;
            for (int j = 0; j < nx; ++j) S = S + w[j];
            for (int d = 0; d < 3; ++d) {
                double num = 0.0;
                for (int j = 0; j < nx; ++j) num = num + w[j] * sj[(size_t)j * 3 + d];
                score_out[d] = num / S;
            }
        }
    }
    free(sj); free(sjs);
    free(x); free(xs); free(lw); free(a); free(w); free(qq); free(anc);
    return ll;
}

double or_pf_loglik(const or_config* cfg, const double* theta, const int32_t* y, int T, int nx,
                    uint64_t seed, uint32_t filt, uint32_t k, double* inc_out, int32_t* rs_out)
{
    return or_pf_trace_state(cfg, theta, y, T, nx, seed, filt, k, inc_out, rs_out, NULL);
}

double or_pf_trace_state(const or_config* cfg, const double* theta, const int32_t* y, int T, int nx,
                         uint64_t seed, uint32_t filt, uint32_t k, double* inc_out, int32_t* rs_out,
                         int32_t* state_out)
{
    return or_pf_trace_full(cfg, theta, y, T, nx, seed, filt, k, inc_out, rs_out, state_out, NULL);
}

double or_pf_trace_full(const or_config* cfg, const double* theta, const int32_t* y, int T, int nx,
                        uint64_t seed, uint32_t filt, uint32_t k, double* inc_out, int32_t* rs_out,
                        int32_t* state_out, int32_t* anc_out)
{
    if (cfg->prec == OR_PREC_FP32)
        return pf_f32(cfg, theta, y, T, nx, seed, filt, k, inc_out, rs_out, state_out, anc_out, NULL);
    return pf_f64(cfg, theta, y, T, nx, seed, filt, k, inc_out, rs_out, state_out, anc_out, NULL);
}

double or_pf_score(const or_config* cfg, const double* theta, const int32_t* y, int T, int nx, uint64_t seed,
                   uint32_t filt, uint32_t k, double* score_out)
{
    if (cfg->model != OR_SIR && cfg->model != OR_SEIR) {
        for (int d = 0; d < cfg->D; ++d) score_out[d] = NAN;
        return NAN;
    }
    if (cfg->prec == OR_PREC_FP32)
        return pf_f32(cfg, theta, y, T, nx, seed, filt, k, NULL, NULL, NULL, NULL, score_out);
    return pf_f64(cfg, theta, y, T, nx, seed, filt, k, NULL, NULL, NULL, NULL, score_out);
}

/*
 * The log-likelihood estimate of one filter recomputed in FP64 from another
 * implementation's integer decisions (Sec. II, injected trajectory):
 *   state[t][c][j]  counts of particle j after day t+1's transitions, before resampling
 *   anc[t][j]       ancestor of slot j after day t+1 (read only where rs[t] = 1)
 *   rs[t]           1 where the filter resampled after day t+1
 * The count each observation looks at follows from a particle's counts and those it
 * started the day from (x_0, or the previous day's counts of its ancestor): the new
 * cases leave S (SIR) or S + E (SEIR models) and nothing else does. Weights,
 * increments and the mean-weight reset after resampling are those of the filter, in
 * FP64. inc_out (may be NULL) receives the per-day increments. Returns the
 * log-likelihood, -inf when every weight vanishes.
 */
double or_pf_replay(const or_config* cfg, const double* th, const int32_t* y, int T, int nx,
                    const int32_t* state, const int32_t* anc, const int32_t* rs, double* inc_out)
{
    const int nc = (cfg->model == OR_SIR) ? 2 : (cfg->model == OR_SEIR ? 3 : 12);
    const int ng = or_n_obs(cfg->model);
    int32_t x0[12];
    const double r = or_model_start(cfg, th, x0);
    double* lw = (double*)malloc(sizeof(double) * (size_t)nx);
    double* a = (double*)malloc(sizeof(double) * (size_t)nx);
    double* w = (double*)malloc(sizeof(double) * (size_t)nx);
    uint64_t* qq = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nx);
    int32_t* unused = (int32_t*)malloc(sizeof(int32_t) * (size_t)nx);
    for (int j = 0; j < nx; ++j) lw[j] = 0.0;
    double s_prev = (double)nx, ll = 0.0;
    for (int t = 0; t < T; ++t) {
        const int32_t* cur = state + (size_t)t * nc * nx;
        double cst = 0.0;
        for (int g = 0; g < ng; ++g) cst = cst + or_obs_const(cfg->obs, y[t * ng + g], r);
        for (int j = 0; j < nx; ++j) {
            int32_t prev[12];
            const int from = (t > 0 && rs[t - 1]) ? anc[(size_t)(t - 1) * nx + j] : j;
            for (int c = 0; c < nc; ++c) prev[c] = t == 0 ? x0[c] : state[((size_t)(t - 1) * nc + c) * nx + from];
            double lg = 0.0;
            for (int g = 0; g < ng; ++g) {
                int32_t cnt;
                if (cfg->model == OR_SIR)
                    cnt = cfg->obs == OR_OBS_POIS_PREV ? cur[1 * nx + j] : prev[0] - cur[0 * nx + j];
                else if (cfg->obs == OR_OBS_POIS_PREV)
                    cnt = cur[(3 * g + 2) * nx + j];
                else
                    cnt = (prev[3 * g] + prev[3 * g + 1]) - (cur[(3 * g) * nx + j] + cur[(3 * g + 1) * nx + j]);
                lg = lg + or_obs_part(cfg->obs, y[t * ng + g], cnt, r);
            }
            a[j] = lw[j] + lg;
        }
        double inc;
        const int st = weigh_f64(nx, a, lw, w, qq, unused, &s_prev, cst, 0, 0, OR_RS_SYSTEMATIC, 0, 0, 0, &inc);
        if (inc_out) inc_out[t] = inc;
        if (st < 0) {
            ll = -INFINITY;
            break;
        }
        ll = ll + inc;
        if (rs[t]) {
            for (int j = 0; j < nx; ++j) lw[j] = 0.0;
            s_prev = (double)nx;
        }
    }
    free(lw); free(a); free(w); free(qq); free(unused);
    return ll;
}

/* ------------------------------------------------------------------ outer sampler */

static double logsumexp(int n, const double* v)
{
    double m = -INFINITY;
    for (int i = 0; i < n; ++i)
        if (v[i] > m) m = v[i];
    if (m == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += exp(v[i] - m);
    return m + log(s);
}

#include "mlp.inc"

/*
 * One outer update at iteration k, given the proposals phi_new with their prior
 * log-densities and particle-filter log-likelihoods:
 *   k = 1:  log w = ll_new                                   (Sec. IV-A, Eq. init_weights)
 *   k > 1:  log w = log w_{k-1} + log pi(new) - log pi(old) + log L - log q
 *                                                            (Sec. IV-A, Eq. l_weights)
 * with pi = prior x likelihood estimate (pseudo-marginal: the estimate travels with
 * its sample). Then normalisation (Eq. normalise_smc2), the estimate (Eq.
 * realised_estimates), l_k = (sum w)^2 / sum w^2 (Eq. recycling_I) = ESS (Eq.
 * ess_smc2), and, if ESS < N/2, systematic resampling with redistribution and reset
 * (Sec. IV-B). The state arrays (phi, lp, ll, logw) are replaced by the new
 * population. logq (may be NULL: the random walk, whose density the function
 * evaluates) holds log q(phi_new | phi) of a learned proposal. L is the fitted
 * Gaussian kernel, or the random walk's Gaussian read backwards when the forward
 * kernel is configured or the fit is rejected (a normalised density in phi_{k-1}
 * for any proposal; for the random walk it cancels q exactly). Records carry, after
 * the estimates, the proposal used (0 random walk, 1 learned) and a slot for the
 * caller (the learned proposal's held-out score). Returns 0, or -4 when every
 * weight is zero.
 */
int or_outer_update(const or_config* cfg, int N, uint32_t k, uint64_t seed,
                    double* phi, double* lp, double* ll, double* logw,
                    const double* phi_new, const double* lp_new, const double* ll_new,
                    const double* logq, double* logw_pre, int32_t* anc, double* rec)
{
    const int D = cfg->D;
    int fallback = 0;
    if (k == 1) {
        for (int i = 0; i < N; ++i) logw_pre[i] = ll_new[i];
    } else {
        /* log L - log q per sample. L is the approximately optimal Gaussian kernel when
           it is configured and its fit succeeds; otherwise (the forward-kernel setting,
           or a rejected fit) it is the random walk's Gaussian read backwards,
           L(phi_{k-1} | phi_k) = N(phi_{k-1}; phi_k, Sigma_RW), a normalised density in
           phi_{k-1} whatever proposal drew phi_k. For the random walk that is its own
           forward kernel (Sec. IV-D), log L - log q is exactly 0, and the weight is the
           target ratio of Eq. aimplified_l_weights; for the learned proposal the
           network's density stays in the weight. */
        double* logL = (double*)calloc((size_t)N, sizeof(double));
        double C[OR_DMAX * OR_DMAX], Lq[OR_DMAX * OR_DMAX];
        for (int a = 0; a < D; ++a)
            for (int c = 0; c < D; ++c) C[a * D + c] = cfg->rw_cov[a][c];
        or_cholesky(D, C, Lq);
        int fit = 0;
        double mu[2 * OR_DMAX], A[OR_DMAX * OR_DMAX], LS[OR_DMAX * OR_DMAX];
        if (cfg->lkernel == OR_L_GAUSS_OPT) {
            double* omega = (double*)malloc(sizeof(double) * (size_t)N);
            double W0 = logsumexp(N, logw);
            for (int i = 0; i < N; ++i) omega[i] = exp(logw[i] - W0);
            fit = or_lkernel_fit(N, D, phi, phi_new, omega, mu, A, LS) == 0;
            fallback = !fit;
            free(omega);
        }
        for (int i = 0; i < N; ++i) {
            const double* xo = phi + (size_t)i * D;
            const double* xn = phi_new + (size_t)i * D;
            double lL;
            if (fit) {
                double m[OR_DMAX];
                for (int a = 0; a < D; ++a) {
                    double s = mu[a];
                    for (int c = 0; c < D; ++c) s += A[a * D + c] * (xn[c] - mu[D + c]);
                    m[a] = s;
                }
                lL = or_mvn_logpdf_chol(D, xo, m, LS);
            } else {
                lL = or_mvn_logpdf_chol(D, xo, xn, Lq);
            }
            double lq = logq ? logq[i] : or_mvn_logpdf_chol(D, xn, xo, Lq);
            logL[i] = lL - lq;
        }
        for (int i = 0; i < N; ++i) {
            double pin = lp_new[i] + ll_new[i];
            if (logw[i] == -INFINITY || pin == -INFINITY) {
                logw_pre[i] = -INFINITY;
            } else {
                double v = (logw[i] + pin) - (lp[i] + ll[i]);
                logw_pre[i] = v + logL[i];
            }
        }
        free(logL);
    }

    /* normalise, ESS, estimates */
    const int RL = or_record_len(D);
    for (int a = 0; a < RL; ++a) rec[a] = 0.0;
    rec[0] = (double)k;
    rec[4] = (double)fallback;
    int n_dead = 0;
    for (int i = 0; i < N; ++i) n_dead += (logw_pre[i] == -INFINITY);
    rec[3] = (double)n_dead;
    double W = logsumexp(N, logw_pre);
    rec[5] = W;
    for (int i = 0; i < N; ++i) anc[i] = i;
    if (W == -INFINITY) {
        for (int i = 0; i < N; ++i) logw[i] = -INFINITY;
        return -4;
    }
    double* wn = (double*)malloc(sizeof(double) * (size_t)N);
    double s2 = 0.0;
    for (int i = 0; i < N; ++i) {
        wn[i] = exp(logw_pre[i] - W);
        s2 += wn[i] * wn[i];
    }
    rec[1] = 1.0 / s2;
    double* mth = rec + 6;
    double* cth = rec + 6 + D;
    double* mph = rec + 6 + D + D * D;
    double th[OR_DMAX];
    for (int i = 0; i < N; ++i) {
        or_theta_of_phi(cfg, phi_new + (size_t)i * D, th);
        for (int a = 0; a < D; ++a) {
            mth[a] += wn[i] * th[a];
            mph[a] += wn[i] * phi_new[i * D + a];
        }
    }
    for (int i = 0; i < N; ++i) {
        or_theta_of_phi(cfg, phi_new + (size_t)i * D, th);
        for (int a = 0; a < D; ++a)
            for (int c = 0; c < D; ++c) cth[a * D + c] += wn[i] * (th[a] - mth[a]) * (th[c] - mth[c]);
    }

    /* resampling (Sec. IV-B) */
    double M = -INFINITY;
    for (int i = 0; i < N; ++i)
        if (logw_pre[i] > M) M = logw_pre[i];
    uint64_t* q = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    for (int i = 0; i < N; ++i) q[i] = (uint64_t)floor(exp(logw_pre[i] - M) * 4294967296.0);
    int rs = or_resample_trigger(q, N);
    rec[2] = (double)rs;
    if (rs) {
        uint32_t ctr[4] = {0u, 0u, k << 16, (uint32_t)OR_S_OUTER_RS << 24};
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t wd[4];
        or_philox(ctr, key, wd);
        or_resample_ancestors(q, N, (uint64_t)wd[0] | ((uint64_t)wd[1] << 32), anc);
    }
    for (int i = 0; i < N; ++i) {
        int s = anc[i];
        for (int a = 0; a < D; ++a) phi[i * D + a] = phi_new[s * D + a];
        lp[i] = lp_new[s];
        ll[i] = ll_new[s];
        logw[i] = rs ? 0.0 : logw_pre[i];
    }
    free(q);
    free(wn);
    return 0;
}

/* ------------------------------------------------------------------ p-MCMC
 * Particle marginal Metropolis-Hastings (Sec. III, after Andrieu, Doucet and Holenstein):
 * a random-walk Metropolis-Hastings chain on the sampler coordinates whose target density
 * uses the particle filter's likelihood estimate. The estimate of the current state is
 * kept until a proposal is accepted (the estimate travels with its state), which makes the
 * chain target the exact posterior for any number of particles. With the symmetric random
 * walk the proposal densities of Eq. MHalgorithm_ cancel. A proposal outside the prior's
 * support is rejected without running its filter.
 * Random numbers (Philox, key = the seed): the chain's starting point, coordinate d,
 * from (c, 0, 0, 11<<24 | d) as the SMC^2 prior draw; at iteration m >= 1 the random-walk
 * normal of coordinate d from (c, 0, m<<16, 9<<24 | d) and the uniform u53 of the words
 * (0, 1) of (c, 0, m<<16, 10<<24); the filter of chain c at iteration m runs on the
 * particle-filter streams of filter c and iteration index m (m = 0: the starting point). */
int or_mh_accept(double lp, double ll, double lp_new, double ll_new, double u)
{
    const double cur = lp + ll, nw = lp_new + ll_new;
    if (nw == -INFINITY) return 0;
    if (cur == -INFINITY) return 1;
    return log(u) < nw - cur;
}

static void or_mcmc_start(const or_config* cfg, uint64_t seed, uint32_t c, double* phi)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int d = 0; d < cfg->D; ++d) {
        const uint32_t ctr[4] = {c, 0u, 0u, ((uint32_t)OR_S_MCMC_INIT << 24) | (uint32_t)d};
        uint32_t w[4];
        or_philox(ctr, key, w);
        const double u1 = or_u53(w[0], w[1]), u2 = or_u53(w[2], w[3]);
        const int fam = (int)cfg->prior[d][0];
        const double a = cfg->prior[d][1], b = cfg->prior[d][2];
        if (fam == OR_PRIOR_UNIFORM) phi[d] = a + (b - a) * u1;
        else phi[d] = a + b * (sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
    }
}

int or_pmcmc_run(const or_config* cfg, const int32_t* y, int T, int nx, uint64_t seed, int chains, int iters,
                 int n_threads, double* theta_trace, double* ll_trace, int32_t* acc_trace)
{
    const int D = cfg->D;
    double C[OR_DMAX * OR_DMAX], L[OR_DMAX * OR_DMAX];
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) C[a * D + b] = cfg->rw_cov[a][b];
    if (or_cholesky(D, C, L) != 0) return -1;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < chains; ++c) {
        double phi[OR_DMAX], phn[OR_DMAX], th[OR_DMAX];
        or_mcmc_start(cfg, seed, (uint32_t)c, phi);
        double lp = or_prior_logpdf(cfg, phi), ll = -INFINITY;
        if (lp != -INFINITY) {
            or_theta_of_phi(cfg, phi, th);
            ll = or_pf_loglik(cfg, th, y, T, nx, seed, (uint32_t)c, 0u, NULL, NULL);
        }
        for (int m = 0; m <= iters; ++m) {
            if (m > 0) {
                double z[OR_DMAX];
                for (int d = 0; d < D; ++d) {
                    const uint32_t ctr[4] = {(uint32_t)c, 0u, (uint32_t)m << 16, ((uint32_t)OR_S_MCMC_RW << 24) | (uint32_t)d};
                    z[d] = or_normal_call(seed, ctr);
                }
                for (int d = 0; d < D; ++d) {
                    double acc = 0.0;
                    for (int e = 0; e <= d; ++e) acc += L[d * D + e] * z[e];
                    phn[d] = phi[d] + acc;
                }
                const double lpn = or_prior_logpdf(cfg, phn);
                double lln = -INFINITY;
                if (lpn != -INFINITY) {
                    or_theta_of_phi(cfg, phn, th);
                    lln = or_pf_loglik(cfg, th, y, T, nx, seed, (uint32_t)c, (uint32_t)m, NULL, NULL);
                }
                const uint32_t ctr[4] = {(uint32_t)c, 0u, (uint32_t)m << 16, (uint32_t)OR_S_MCMC_U << 24};
                uint32_t w[4];
                or_philox(ctr, key, w);
                const int acc = or_mh_accept(lp, ll, lpn, lln, or_u53(w[0], w[1]));
                if (acc) {
                    for (int d = 0; d < D; ++d) phi[d] = phn[d];
                    lp = lpn;
                    ll = lln;
                }
                if (acc_trace) acc_trace[(size_t)c * iters + (m - 1)] = acc;
            }
            if (theta_trace) {
                or_theta_of_phi(cfg, phi, th);
                for (int d = 0; d < D; ++d) theta_trace[((size_t)c * (iters + 1) + m) * D + d] = th[d];
            }
            if (ll_trace) ll_trace[(size_t)c * (iters + 1) + m] = ll;
        }
    }
    return 0;
}

/* Recycled estimate (Sec. IV-C): c_k = l_k / sum l, mean = sum c_k f_k; the covariance
 * combines the per-iteration second moments with the same constants. */
void or_recycle(int K, int D, const double* rec, double* mean, double* cov, double* c_out)
{
    const int RL = or_record_len(D);
    double lsum = 0.0;
    for (int k = 0; k < K; ++k) lsum += rec[k * RL + 1];
    for (int a = 0; a < D; ++a) mean[a] = 0.0;
    for (int a = 0; a < D * D; ++a) cov[a] = 0.0;
    for (int k = 0; k < K; ++k) {
        double c = rec[k * RL + 1] / lsum;
        if (c_out) c_out[k] = c;
        const double* m = rec + k * RL + 6;
        const double* C = rec + k * RL + 6 + D;
        for (int a = 0; a < D; ++a) mean[a] += c * m[a];
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) cov[a * D + b] += c * (C[a * D + b] + m[a] * m[b]);
    }
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) cov[a * D + b] -= mean[a] * mean[b];
}

/*
 * A whole SMC^2 run (Sec. IV): K iterations over N samples, each sample's
 * likelihood estimated by a particle filter with nx particles. Per-iteration dumps
 * (pre-resampling proposals, their log-likelihoods, log-priors, log-weights and the
 * ancestors chosen) are written when the pointers are not NULL; each holds K
 * consecutive blocks. Returns 0, or the first non-zero status of an update; -5 for a
 * model the reference sampler does not run (only the epidemic models: the
 * linear-Gaussian filter is or_pf_lg, on real observations).
 */
int or_smc2_run(const or_config* cfg, const int32_t* y, int T, int nx, uint64_t seed, int N, int K,
                int n_threads, double* rec, double* phi_dump, double* ll_dump, double* lp_dump,
                double* logw_dump, int32_t* anc_dump)
{
    if (cfg->model != OR_SIR && cfg->model != OR_SEIR && cfg->model != OR_AGE_SEIR) return -5;
    const int D = cfg->D;
    const int RL = or_record_len(D);
    double* phi = (double*)calloc((size_t)N * D, sizeof(double));
    double* lp = (double*)calloc((size_t)N, sizeof(double));
    double* ll = (double*)calloc((size_t)N, sizeof(double));
    double* logw = (double*)calloc((size_t)N, sizeof(double));
    double* phin = (double*)calloc((size_t)N * D, sizeof(double));
    double* lpn = (double*)calloc((size_t)N, sizeof(double));
    double* lln = (double*)calloc((size_t)N, sizeof(double));
    double* lwp = (double*)calloc((size_t)N, sizeof(double));
    int32_t* anc = (int32_t*)calloc((size_t)N, sizeof(int32_t));
    double* lq = (double*)calloc((size_t)N, sizeof(double));
    const int mlp = cfg->proposal == OR_PROP_MLP;
    const int lgv = cfg->proposal == OR_PROP_LANGEVIN;
    const int rwp = cfg->proposal == OR_PROP_RW_POP;
    /* Langevin: the score estimates of the population and of the proposals */
    double* sc = lgv ? (double*)calloc((size_t)N * D, sizeof(double)) : NULL;
    double* scn = lgv ? (double*)calloc((size_t)N * D, sizeof(double)) : NULL;
    const int np = or_mlp_nparams(D);
    float* params = mlp ? (float*)calloc((size_t)np, sizeof(float)) : NULL;
    float* am = mlp ? (float*)calloc((size_t)np, sizeof(float)) : NULL;
    float* av = mlp ? (float*)calloc((size_t)np, sizeof(float)) : NULL;
    int32_t adam_t = 0;
    double frame[OR_DMAX + OR_DMAX * OR_DMAX];
    int use_mlp = 0;
    if (mlp) or_mlp_init(D, seed, params);
    int status = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    for (int k = 1; k <= K; ++k) {
        const int learned = (k > 1) && use_mlp;
        if (k == 1) {
            or_prior_draw(cfg, N, seed, phin, lpn);
        } else if (learned) {
            for (int i = 0; i < N; ++i) {
                double u[OR_DMAX], h1[OR_MLP_H], h2[OR_MLP_H], o[OR_DMAX + OR_DMAX * (OR_DMAX + 1) / 2];
                mlp_whiten(D, frame, phi + (size_t)i * D, u);
                or_mlp_forward(D, params, u, 1, h1, h2, o);
                lq[i] = or_mlp_propose_one(D, frame, o, seed, (uint32_t)k, i, phin + (size_t)i * D);
                lpn[i] = or_prior_logpdf(cfg, phin + (size_t)i * D);
            }
        } else if (lgv || rwp) {
            /* the proposal covariance: the weighted covariance of the proposing population
               (its Cholesky factor as the learned proposal's frame forms it) */
            const double Wl = logsumexp(N, logw);
            double* wn = (double*)malloc(sizeof(double) * (size_t)N);
            for (int i = 0; i < N; ++i) wn[i] = exp(logw[i] - Wl);
            double fr[OR_DMAX + OR_DMAX * OR_DMAX];
            or_mlp_frame(N, D, phi, wn, fr);
            free(wn);
            for (int i = 0; i < N; ++i) {
                if (lgv) {
                    lq[i] = or_propose_langevin_one(cfg, fr + D, phi + (size_t)i * D, sc + (size_t)i * D, seed,
                                                    (uint32_t)k, i, phin + (size_t)i * D);
                } else { /* the random walk with the population's covariance: phi' = phi + F z */
                    const double* ph = phi + (size_t)i * D;
                    const double* F = fr + D;
                    double z[OR_DMAX];
                    for (int d = 0; d < D; ++d) {
                        uint32_t ctr[4] = {(uint32_t)i, 0u, (uint32_t)k << 16, ((uint32_t)OR_S_RW << 24) | (uint32_t)d};
                        z[d] = or_normal_call(seed, ctr);
                    }
                    for (int a = 0; a < D; ++a) {
                        double acc = 0.0;
                        for (int c = 0; c <= a; ++c) acc += F[a * D + c] * z[c];
                        phin[(size_t)i * D + a] = ph[a] + acc;
                    }
                    lq[i] = or_mvn_logpdf_chol(D, phin + (size_t)i * D, ph, F);
                }
                lpn[i] = or_prior_logpdf(cfg, phin + (size_t)i * D);
            }
        } else {
            or_propose_rw(cfg, N, seed, (uint32_t)k, phi, phin, lpn);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int i = 0; i < N; ++i) {
            int run = (k == 1) || (logw[i] != -INFINITY && lpn[i] != -INFINITY);
            if (run) {
                double th[OR_DMAX];
                or_theta_of_phi(cfg, phin + (size_t)i * D, th);
                if (lgv)
                    lln[i] = or_pf_score(cfg, th, y, T, nx, seed, (uint32_t)i, (uint32_t)k, scn + (size_t)i * D);
                else
                    lln[i] = or_pf_loglik(cfg, th, y, T, nx, seed, (uint32_t)i, (uint32_t)k, NULL, NULL);
            } else {
                lln[i] = -INFINITY;
                if (lgv)
                    for (int d = 0; d < D; ++d) scn[(size_t)i * D + d] = 0.0;
            }
        }
        double* rk = rec + (size_t)(k - 1) * RL;
        const int drift = (lgv || rwp) && k > 1; /* proposals with their own density in lq */
        int st = or_outer_update(cfg, N, (uint32_t)k, seed, phi, lp, ll, logw, phin, lpn, lln,
                                 (learned || drift) ? lq : NULL, lwp, anc, rk);
        rk[RL - 2] = learned ? 1.0 : (drift ? (lgv ? 2.0 : 3.0) : 0.0);
        if (lgv && st == 0) /* the scores travel with their samples through resampling */
            for (int i = 0; i < N; ++i)
                for (int d = 0; d < D; ++d) sc[(size_t)i * D + d] = scn[(size_t)anc[i] * D + d];
        if (mlp && st == 0) {
            double nm, nr;
            use_mlp = or_mlp_train(cfg, N, phi, logw, seed, (uint32_t)k, cfg->mlp_epochs, cfg->mlp_batch, cfg->mlp_lr,
                                   params, am, av, &adam_t, frame, &nm, &nr);
            rk[RL - 1] = nm - nr;
        }
        if (phi_dump) memcpy(phi_dump + (size_t)(k - 1) * N * D, phin, sizeof(double) * (size_t)N * D);
        if (ll_dump) memcpy(ll_dump + (size_t)(k - 1) * N, lln, sizeof(double) * (size_t)N);
        if (lp_dump) memcpy(lp_dump + (size_t)(k - 1) * N, lpn, sizeof(double) * (size_t)N);
        if (logw_dump) memcpy(logw_dump + (size_t)(k - 1) * N, lwp, sizeof(double) * (size_t)N);
        if (anc_dump) memcpy(anc_dump + (size_t)(k - 1) * N, anc, sizeof(int32_t) * (size_t)N);
        if (st != 0) {
            status = st;
            break;
        }
    }
    free(phi); free(lp); free(ll); free(logw); free(phin); free(lpn); free(lln); free(lwp); free(anc);
    free(lq); free(params); free(am); free(av); free(sc); free(scn);
    return status;
}
