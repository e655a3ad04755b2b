/*
 * smc2_oracle.h — plain CPU reference of the SMC^2 sampler (test infrastructure only).
 *
 * This library exists to check the GPU implementation. Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it. It shares no code,
 * header, table or constant generator with the GPU library: both sides implement the
 * same published definitions (the paper's equations plus the conventions written in
 * the comments of smc2_oracle.c) independently.
 *
 * Paper: Rosato, Varsi, Murphy, Maskell, "An O(log2 N) SMC^2 Algorithm on Distributed
 * Memory with an Approx. Optimal L-Kernel" (arXiv 2311.12973).
 *   - particle filter: Sec. II (weight recursion, likelihood estimate, ESS, resampling)
 *   - SMC^2 outer sampler: Sec. IV-A (IS, RW proposal, weight update, recycling),
 *     Sec. IV-B (ESS, systematic resampling, Alg. 1), Sec. IV-D (L-kernels)
 *   - SIR model: Sec. V-A.
 *
 * All floating-point outside the particle filter is FP64. The particle filter runs
 * in the precision selected by `prec` (OR_PREC_FP32 or OR_PREC_FP64); the cross-time
 * log-likelihood accumulation is FP64 in both.
 */
#ifndef SMC2_ORACLE_H
#define SMC2_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_SIR = 0, OR_SEIR = 1, OR_AGE_SEIR = 2 };
enum { OR_OBS_POIS_PREV = 0, OR_OBS_POIS_INC = 1, OR_OBS_NB_INC = 2 };
enum { OR_PREC_FP32 = 0, OR_PREC_FP64 = 1 };
enum { OR_PRIOR_UNIFORM = 0, OR_PRIOR_LOGNORMAL = 1, OR_PRIOR_LOGITNORMAL = 2, OR_PRIOR_NORMAL = 3 };
enum { OR_L_FORWARD = 0, OR_L_GAUSS_OPT = 1 };
enum { OR_PROP_RW = 0, OR_PROP_MLP = 1, OR_PROP_LANGEVIN = 2, OR_PROP_RW_POP = 3 };

/* Philox stream identifiers (bits 24..31 of the fourth counter word). */
enum { OR_S_PF_PROP = 1, OR_S_PF_RS = 2, OR_S_PRIOR = 3, OR_S_RW = 4, OR_S_OUTER_RS = 5,
       OR_S_MLP_INIT = 6, OR_S_MLP_PERM = 7, OR_S_MCMC_RW = 9, OR_S_MCMC_U = 10, OR_S_MCMC_INIT = 11 };

#define OR_DMAX 8

/* particle-filter resampling schemes */
enum { OR_RS_SYSTEMATIC = 0, OR_RS_MULTINOMIAL = 1 };

/* Event counters of the particle filter (see or_events_get). */
enum { OR_EV_PSTEP = 0, OR_EV_DRAW, OR_EV_PHILOX, OR_EV_INV, OR_EV_INV_ITER, OR_EV_BTRS, OR_EV_ATTEMPT,
       OR_EV_FINAL, OR_EV_T64, OR_EV_RS_PARTICLE, OR_EV_N };
/* relative numerical-rank floor of the L-kernel fit (see or_lkernel_fit) */
#define OR_LK_REL_FLOOR 1e-12
#define OR_NFIXED 32

typedef struct {
    int32_t model, obs, D, prec;
    int32_t pf_always;  /* 1: resample the particle filter at every step; 0: when ESS < Nx/2 */
    int32_t lkernel;    /* OR_L_FORWARD or OR_L_GAUSS_OPT */
    int32_t proposal;   /* OR_PROP_RW, OR_PROP_MLP, OR_PROP_LANGEVIN or OR_PROP_RW_POP */
    int32_t n_fixed;
    double n_pop;
    double prior[OR_DMAX][3];      /* {family, a, b} per sampler coordinate */
    double rw_cov[OR_DMAX][OR_DMAX];
    double fixed[OR_NFIXED];       /* model constants (see smc2_oracle.c, "Models") */
    int32_t mlp_epochs, mlp_batch; /* learned proposal: epochs and minibatch rows per iteration */
    double mlp_lr;                 /* learned proposal: Adam learning rate */
    int32_t pf_resampling;         /* OR_RS_SYSTEMATIC or OR_RS_MULTINOMIAL (the particle filter's) */
    int32_t pad;
    double lgv_step;               /* Langevin proposal: the fraction of the truncated drift
                                      applied, in (0, 1]; 0 selects 1/4 */
} or_config;

/* Number of doubles in one per-iteration record. */
int or_record_len(int D);
int or_n_obs(int model);

/* ---- building blocks (exported for the pins) ---- */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float or_u24(uint32_t x);
double or_u53(uint32_t lo, uint32_t hi);
double or_normal_call(uint64_t seed, const uint32_t ctr[4]);
/* One binomial draw at particle-filter coordinates (j, i, k, t, b). p is rounded to
 * the working precision first when prec == OR_PREC_FP32. */
int32_t or_binomial(int prec, int32_t n, double p, uint64_t seed, uint32_t j, uint32_t i,
                    uint32_t k, uint32_t t, uint32_t b);
void or_binomial_batch(int prec, int32_t n, double p, uint64_t seed, uint32_t i, uint32_t k,
                       uint32_t t, uint32_t b, int count, int32_t* out);
void or_binomial_many(int prec, int count, const int32_t* n, const double* p, uint64_t seed, uint32_t i,
                      uint32_t k, uint32_t t, uint32_t b, int32_t* out);
double or_obs_logpmf(int obs, int32_t y, int32_t count, double r);
int or_resample_trigger(const uint64_t* q, int n);
void or_resample_ancestors(const uint64_t* q, int n, uint64_t x64, int32_t* anc);
int or_cholesky(int n, const double* A, double* L);
double or_mvn_logpdf_chol(int n, const double* x, const double* mu, const double* L);
int or_lkernel_fit(int N, int D, const double* phi, const double* phi_new, const double* omega,
                   double* mu /*2D*/, double* A /*DxD*/, double* LS /*DxD*/);
/* As or_lkernel_fit, also writing the fitted 2D x 2D weighted covariance (cov_out, may
 * be NULL); the moments are written even when the conditioning is rejected. */
int or_lkernel_fit_cov(int N, int D, const double* phi, const double* phi_new, const double* omega,
                       double* mu, double* A, double* LS, double* cov_out);
double or_prior_logpdf(const or_config* cfg, const double* phi);
void or_theta_of_phi(const or_config* cfg, const double* phi, double* theta);
void or_recycle(int K, int D, const double* rec, double* mean, double* cov, double* c_out);

/* ---- the particle filter (Sec. II) ---- */
double or_pf_loglik(const or_config* cfg, const double* theta, const int32_t* y, int T, int nx,
                    uint64_t seed, uint32_t filt, uint32_t k, double* inc_out, int32_t* rs_out);

/* As or_pf_loglik, also writing every day's particle counts before resampling
 * (state_out: int32[T][n_counts][nx], n_counts = 2 / 3 / 12 for SIR / SEIR / age). */
double or_pf_trace_state(const or_config* cfg, const double* theta, const int32_t* y, int T, int nx,
                         uint64_t seed, uint32_t filt, uint32_t k, double* inc_out, int32_t* rs_out,
                         int32_t* state_out);
/* As or_pf_trace_state, also writing the ancestors chosen after every day (anc_out:
 * int32[T][nx], the identity on days without resampling; may be NULL). */
double or_pf_trace_full(const or_config* cfg, const double* theta, const int32_t* y, int T, int nx,
                        uint64_t seed, uint32_t filt, uint32_t k, double* inc_out, int32_t* rs_out,
                        int32_t* state_out, int32_t* anc_out);
/* The FP64 log-likelihood estimate of a filter replayed from injected integer decisions:
 * state int32[T][n_counts][nx] and anc int32[T][nx] as or_pf_trace_full writes them,
 * rs int32[T] resampling flags; inc_out (T, optional) the per-day increments. */
double or_pf_replay(const or_config* cfg, const double* theta, const int32_t* y, int T, int nx,
                    const int32_t* state, const int32_t* anc, const int32_t* rs, double* inc_out);

/* ---- particle marginal Metropolis-Hastings (Sec. III), the paper's comparison ----
 * `chains` independent chains of `iters` random-walk Metropolis-Hastings iterations each;
 * theta_trace [chains][iters+1][D] (state 0: the prior draw the chain starts from),
 * ll_trace [chains][iters+1], acc_trace [chains][iters] (may each be NULL). */
int or_pmcmc_run(const or_config* cfg, const int32_t* y, int T, int nx, uint64_t seed, int chains, int iters,
                 int n_threads, double* theta_trace, double* ll_trace, int32_t* acc_trace);
/* The Metropolis-Hastings decision of Eq. MHalgorithm_ for a symmetric proposal, from
 * the log prior and log-likelihood estimate of the current and proposed states and the
 * uniform u in (0, 1): accept when the proposal has positive target and either the
 * current state has none or log u < (lp_new + ll_new) - (lp + ll). */
int or_mh_accept(double lp, double ll, double lp_new, double ll_new, double u);

/* ---- the outer sampler (Sec. IV) ---- */
void or_prior_draw(const or_config* cfg, int N, uint64_t seed, double* phi, double* lp);
void or_propose_rw(const or_config* cfg, int N, uint64_t seed, uint32_t k, const double* phi,
                   double* phi_new, double* lp_new);
int or_outer_update(const or_config* cfg, int N, uint32_t k, uint64_t seed,
                    double* phi, double* lp, double* ll, double* logw,
                    const double* phi_new, const double* lp_new, const double* ll_new,
                    const double* logq, double* logw_pre, int32_t* anc, double* rec);
/* learned proposal (mlp.inc) */
int or_mlp_nout(int D);
int or_mlp_nparams(int D);
void or_mlp_init(int D, uint64_t seed, float* w);
void or_mlp_forward(int D, const float* w, const double* u, int bf16, double* h1, double* h2, double* o);
double or_mlp_nll(int D, const double* o, const double* ut, double* grad);
void or_mlp_backward(int D, const float* w, const double* u, const double* h1, const double* h2, const double* go,
                     int bf16, double* grad);
void or_adam_step(int n, float* p, float* m, float* v, const double* g, int t, double lr);
void or_mlp_perm(uint64_t seed, uint32_t k, uint32_t e, uint32_t which, int N, uint64_t* a, uint64_t* b);
int or_mlp_frame_len(int D);
void or_mlp_frame(int N, int D, const double* phi, const double* wn, double* frame);
int or_mlp_train(const or_config* cfg, int N, const double* phi, const double* logw, uint64_t seed, uint32_t k,
                 int epochs, int batch, double lr, float* params, float* adam_m, float* adam_v, int32_t* adam_t,
                 double* frame, double* nll_mlp, double* nll_rw);
double or_mlp_propose_one(int D, const double* frame, const double* o, uint64_t seed, uint32_t k, int i,
                          double* phi_new);

int or_smc2_run(const or_config* cfg, const int32_t* y, int T, int nx, uint64_t seed, int N, int K,
                int n_threads, double* rec, double* phi_dump, double* ll_dump, double* lp_dump,
                double* logw_dump, int32_t* anc_dump);

/* Totals of the event counters over every particle filter run since the last reset
 * (out[OR_EV_N], indexed by OR_EV_*). */
void or_events_get(double* out);
void or_events_reset(void);

/* Particle filter on a scalar linear-Gaussian model (a pin against the Kalman filter):
 * x_0 ~ N(m0, s0^2), x_t = phi x_{t-1} + sq e_t, y_t = x_t + sr d_t; returns the log of
 * the likelihood estimate; k is the iteration index of the streams; inc_out / rs_out
 * (T entries, optional) as or_pf_loglik; x_out (T x nx, optional) the states of each
 * day before resampling; score_out (3, optional, needs sq > 0) the estimate of the score
 * d log p(y) / d(phi, sq, sr) as or_pf_score forms it. */
double or_pf_lg(double phi, double sq, double sr, double m0, double s0, const double* y, int T, int nx,
                uint64_t seed, uint32_t filt, uint32_t k, int pf_always, int resampling, double* inc_out,
                int32_t* rs_out, double* x_out, double* score_out);

/* Score of the log-likelihood estimate (Fisher's identity: grad log p(y | theta) =
 * E[grad log p(x_{0:T}, y | theta) | y]), estimated by the same filter: each particle
 * carries the running complete-data score of its trajectory on the natural parameters
 * theta (the flows' d log Bin / d theta, and d log NB / d r when r is estimated),
 * resampling moves it with the particle, and the last day's weights average it. SIR and
 * SEIR; the SEIR initial fraction iota enters only through a rounding and gets 0.
 * score_out: D doubles (0 when every weight vanished; NaN for other models). Returns
 * the log-likelihood estimate, equal to or_pf_loglik's. */
double or_pf_score(const or_config* cfg, const double* theta, const int32_t* y, int T, int nx, uint64_t seed,
                   uint32_t filt, uint32_t k, double* score_out);
/* Digamma function psi(x), x > 0. */
double or_digamma(double x);

/* The truncated Langevin proposal of sample phi given the score estimate s_theta (on the
 * natural parameters) that travelled with it: the drift 1/2 Sigma g with
 * g = J s_theta + grad log prior(phi) (J = d theta / d phi per coordinate), shrunk to a
 * Mahalanobis length of at most 1 (|L^-1 . | <= 1, L L' = Sigma), times the step fraction
 * s = cfg->lgv_step (1/4 when 0): delta; phi_new = phi + delta + L z with z the random
 * walk's normals of sample i at iteration k.
 * Returns log q(phi_new | phi) = log N(phi_new; phi + delta, Sigma). The sampler takes
 * Sigma as the weighted covariance of the proposing population (L its frame's factor,
 * or_mlp_frame). */
double or_propose_langevin_one(const or_config* cfg, const double* L, const double* phi, const double* s_theta,
                               uint64_t seed, uint32_t k, int i, double* phi_new);
/* Multinomial ancestors from quantised weights: slot m draws U_m = floor(x64_m Q / 2^64)
 * (x64_m: 64-bit word m&1 of the Philox call (m>>1, filt, kt, 2<<24 | 1<<16)) and takes
 * the first j whose inclusive scan C_j exceeds U_m. */
void or_resample_multinomial(const uint64_t* q, int n, uint64_t seed, uint32_t filt, uint32_t kt, int32_t* anc);

#ifdef __cplusplus
}
#endif
#endif
