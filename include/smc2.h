/*
 * smc2.h — C ABI of the MI355X SMC^2 library (libsmc2.so).
 *
 * The library runs the sampler of Rosato, Varsi, Murphy and Maskell, "An O(log2 N)
 * SMC^2 Algorithm on Distributed Memory with an Approx. Optimal L-Kernel"
 * (arXiv 2311.12973) on one AMD Instinct MI355X (gfx950):
 *
 *   - For every parameter sample theta^i (i < N) a particle filter with N_x particles
 *     estimates the likelihood p(y_{1:T} | theta^i) (Sec. II: weight recursion,
 *     likelihood estimate as the mean unnormalised weight, ESS-triggered resampling
 *     with the mean-weight reset).
 *   - The outer SMC sampler (Sec. IV) draws theta_1 from the prior (Eq. init_sample),
 *     moves theta with a Gaussian random walk (Eq. proposal) or one of the other
 *     proposals below (Sec. IV-A leaves q free), weights with an
 *     L-kernel (Eq. l_weights; forward kernel, Eq. aimplified_l_weights, or the
 *     approximately optimal Gaussian kernel, Eq. Gauss_joint and the conditional that
 *     follows), normalises (Eq. normalise_smc2), estimates (Eq. realised_estimates),
 *     computes l_k (Eq. recycling_I) and ESS (Eq. ess_smc2), resamples
 *     systematically when ESS < N/2 (Eq. cdf, ncopies; Alg. 1 as a prefix-sum
 *     scatter) and recycles the per-iteration estimates (Sec. IV-C).
 *
 * Several independent runs (one data series, seed, T and N_x each, same config)
 * can share one context; each iteration then advances all of them together.
 *
 * Ownership: the caller owns every argument. smc2_init deep-copies the config, the
 * run descriptions and the observations, which may be freed after it returns. The
 * caller also owns the device workspace (at least smc2_workspace_bytes bytes of
 * device memory, 256-byte aligned) and the HIP stream; both must outlive the
 * context. The library never allocates device memory; every device buffer is
 * carved out of the workspace. smc2_destroy frees host state only.
 *
 * Synchronisation: smc2_step enqueues one iteration on the stream and returns
 * without waiting. smc2_estimate, smc2_records and smc2_dump synchronise the stream.
 *
 * Errors: every function returns a status (SMC2_OK = 0 or a negative code) and
 * never throws. Arguments are checked before anything is enqueued. A failed HIP
 * call poisons the context: every later call returns SMC2_E_DEVICE.
 * smc2_last_error gives a message for the last failure of a context (or of the
 * calling thread when ctx is NULL). A context is used by one thread at a time;
 * separate contexts on separate streams are independent.
 */
#ifndef SMC2_H
#define SMC2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SMC2_OK 0
#define SMC2_E_ARG (-1)         /* invalid argument or workspace too small */
#define SMC2_E_DEVICE (-2)      /* a HIP call failed; the context is poisoned */
#define SMC2_E_STATE (-3)       /* call out of order (e.g. more than K steps) */
#define SMC2_E_NUMERIC (-4)     /* every weight of a run is zero */
#define SMC2_E_UNSUPPORTED (-5) /* valid but not supported combination */

/* model (Sec. V-A chain-binomial SIR and its SEIR extensions) */
#define SMC2_SIR 0      /* theta = (beta, gamma); fixed[0] = initially infected I_0 */
#define SMC2_SEIR 1     /* theta = (beta, sigma, gamma, iota[, r]); I_0 = round(iota N_pop);
                           fixed[0] = negative-binomial dispersion r when D == 4 */
#define SMC2_AGE_SEIR 2 /* theta = (beta, sigma, gamma, iota, r, s_2, s_3, s_4), four groups;
                           fixed[0..15] contact matrix (row-major), fixed[16..19] group fractions */
#define SMC2_LINGAUSS 3 /* scalar linear-Gaussian model, a test model whose likelihood the
                           Kalman filter gives in closed form (Sec. II's filter on it is
                           otherwise the epidemic models'): theta = (a, sigma_x, sigma_y),
                           x_t = a x_{t-1} + sigma_x e_t, y_t = x_t + sigma_y d_t, e, d ~ N(0, 1),
                           x_0 = fixed[0] + fixed[1] e_0; real observations (smc2_run.y_real);
                           SMC2_OBS_GAUSS; SMC2_PREC_FP64 only; n_pop is not used             */

/* observation model of y_t */
#define SMC2_OBS_POIS_PREV 0 /* Poisson(I_t)            (Sec. V-A)                      */
#define SMC2_OBS_POIS_INC 1  /* Poisson(new infections) (S->I for SIR, E->I for SEIR)   */
#define SMC2_OBS_NB_INC 2    /* negative binomial(mean = new infections, dispersion r)  */
#define SMC2_OBS_GAUSS 3     /* N(x_t, sigma_y^2) (SMC2_LINGAUSS)                       */

/* precision of the particle-filter propagation and per-step weights. The
 * log-likelihood accumulation and everything in the outer sampler are FP64. */
#define SMC2_PREC_FP32 0
#define SMC2_PREC_FP64 1

/* prior family per sampler coordinate phi_d (the sampler moves on phi) */
#define SMC2_PRIOR_UNIFORM 0     /* theta_d = phi_d ~ U[a, b]                   */
#define SMC2_PRIOR_LOGNORMAL 1   /* theta_d = exp(phi_d),     phi_d ~ N(a, b^2) */
#define SMC2_PRIOR_LOGITNORMAL 2 /* theta_d = logistic(phi_d), phi_d ~ N(a, b^2) */
#define SMC2_PRIOR_NORMAL 3      /* theta_d = phi_d ~ N(a, b^2)                 */

/* L-kernel of Eq. l_weights. Whenever the Gaussian fit is not used (SMC2_L_FORWARD, or
 * a rejected fit, reported in the record) L(phi_{k-1} | phi_k) = N(phi_{k-1}; phi_k,
 * Sigma_RW): for the random walk this is the forward proposal of Sec. IV-D and the
 * weight is the target ratio (Eq. aimplified_l_weights); for the other proposals it is
 * still a normalised density in phi_{k-1}, and their log q stays in the weight. */
#define SMC2_L_FORWARD 0   /* L = the random walk's forward kernel (Sec. IV-D)          */
#define SMC2_L_GAUSS_OPT 1 /* approximately optimal Gaussian L-kernel (Sec. IV-D)       */

#define SMC2_PROP_RW 0  /* Gaussian random walk on phi (Eq. proposal) */
#define SMC2_PROP_MLP 1 /* learned Gaussian proposal: a D -> 64 -> 64 -> (mean, Cholesky)
                           network, BF16 matrix-core products, trained after every
                           iteration on the weighted population; its exact density
                           enters the weights (Eq. l_weights, with either L-kernel);
                           the random walk whenever the network does not beat it on
                           held-out pairs                                                */
#define SMC2_PROP_LANGEVIN 2 /* truncated Langevin proposal (SIR, SEIR, SMC2_LINGAUSS):
                                phi' = phi + delta + L z, Sigma = L L' the weighted covariance
                                of the proposing population, delta = s times 1/2 Sigma g
                                shrunk to Mahalanobis length <= 1 (s = lgv_step, 1/4 by
                                default), g the gradient of log(prior x
                                likelihood) on the sampler coordinates from the filter's
                                score estimate (smc2_pf_score's), which travels with its
                                sample; its exact log q enters the weights (Eq. l_weights) */
#define SMC2_PROP_RW_POP 3 /* random walk with the population's covariance (every model):
                               phi' = phi + L z, Sigma = L L' the weighted covariance of
                               the proposing population (SMC2_PROP_LANGEVIN's covariance,
                               without its drift); its log q enters the weights
                               (Eq. l_weights). Iteration 1 draws from the prior. */

/* particle-filter draw schedule (smc2_config.schedule); both give identical results */
#define SMC2_SCHED_AUTO 0     /* pooled where supported and it fits in LDS, else per draw
                                 (the score launches of SMC2_PROP_LANGEVIN: per draw)     */
#define SMC2_SCHED_PER_DRAW 1 /* each lane finishes its draws one after another          */
#define SMC2_SCHED_POOLED 2   /* SIR/SEIR: a wave pools its draws and runs the final
                                 acceptance tests of the BTRS sampler 64 at a time        */

/* Particle-filter resampling (Sec. II; both from the quantised weights q_j and their
 * inclusive scan C, Q = C_{N_x - 1}, in exact integers):
 *   SYSTEMATIC  one uniform U per filter-step, ancestor of slot m = min{j : N_x C_j > m Q + U}
 *   MULTINOMIAL one uniform U_m per slot, ancestor of slot m = min{j : C_j > U_m}, i.e.
 *               probability q_j / Q independently per slot (the paper's filter)          */
#define SMC2_PF_RS_SYSTEMATIC 0
#define SMC2_PF_RS_MULTINOMIAL 1

/* Training layout of the learned proposal (smc2_config.mlp_train). Per run: one
 * workgroup per run takes every minibatch step. Split: each minibatch's 64-row
 * sub-batches take a workgroup each and a second launch sums their gradients in order
 * and takes the Adam step (for few runs, which would leave most of the device idle).
 * The two group the minibatch's rows differently, so they agree to FP32 rounding. */
#define SMC2_MLP_TRAIN_AUTO 0    /* split for up to 32 runs, per run above               */
#define SMC2_MLP_TRAIN_PER_RUN 1
#define SMC2_MLP_TRAIN_SPLIT 2

/* Particle-filter launch (smc2_config.persistent, with tune = 0; the autotuner chooses
 * for itself). Persistent: the resident workgroups pull filters from the cost-sorted work
 * list (an atomic counter) until it is exhausted. */
#define SMC2_LAUNCH_AUTO 0       /* persistent when a launch group has more filters than
                                    fit on the device at once, else a workgroup per filter */
#define SMC2_LAUNCH_PERSISTENT 1
#define SMC2_LAUNCH_PER_FILTER 2 /* one workgroup per filter                               */

#define SMC2_DMAX 8
#define SMC2_NFIXED 32

typedef struct smc2_ctx smc2_ctx;

typedef struct {
    int32_t model;     /* SMC2_SIR / SMC2_SEIR / SMC2_AGE_SEIR / SMC2_LINGAUSS          */
    int32_t obs;       /* SMC2_OBS_*                                                    */
    int32_t D;         /* number of parameters, 1..SMC2_DMAX (fixed by the model)       */
    int32_t N;         /* parameter samples per run, 2..32768                           */
    int32_t K;         /* iterations, >= 1 (k = 1 is the prior importance-sampling step) */
    int32_t precision; /* SMC2_PREC_FP32 or SMC2_PREC_FP64                              */
    int32_t proposal;  /* SMC2_PROP_RW, _MLP, _LANGEVIN or _RW_POP                       */
    int32_t lkernel;   /* SMC2_L_FORWARD or SMC2_L_GAUSS_OPT                            */
    int32_t pf_always; /* 1: resample the particle filter at every step                 */
    int32_t use_graph; /* 1: replay each iteration as one captured HIP graph            */
    int32_t block;     /* particle-filter workgroup size, a multiple of 64 up to 1024
                          (0: chosen from the filter's LDS footprint)                   */
    int32_t schedule;  /* SMC2_SCHED_*: particle-filter draw schedule (same results)     */
    double n_pop;      /* population size, integer, 1 .. 2^24 (not used by SMC2_LINGAUSS) */
    const double* prior;  /* host, D x 3 row-major: {family, a, b} per coordinate        */
    const double* rw_cov; /* host, D x D row-major, symmetric positive definite          */
    const double* fixed;  /* host, n_fixed model constants (see the model codes)         */
    int32_t n_fixed;
    int32_t tune;       /* 1: smc2_init times the candidate particle-filter launch
                           configurations (workgroup size, draw schedule, persistent grid)
                           of every launch group on a sample of its filters and keeps the
                           fastest; 0: defaults from the LDS footprint. Same results.     */
    int32_t persistent; /* with tune = 0, SMC2_LAUNCH_*: how the filters are launched
                           (same results)                                                 */
    int32_t mlp_epochs; /* learned proposal: training epochs per iteration (0 .. 1000)     */
    int32_t mlp_batch;  /* learned proposal: minibatch rows (0: the whole population)      */
    double mlp_lr;      /* learned proposal: Adam learning rate (> 0)                      */
    int32_t pf_resampling; /* SMC2_PF_RS_*: the particle filters' resampling scheme       */
    int32_t mlp_train;     /* SMC2_MLP_TRAIN_*: how the learned proposal's training is laid
                              out on the device (same mathematics, FP32 rounding aside)   */
    double lgv_step;       /* SMC2_PROP_LANGEVIN: the fraction of the truncated drift
                              applied, in (0, 1]; 0 selects 1/4                           */
} smc2_config;

typedef struct {
    int32_t T;          /* number of observations, 1..1024                             */
    int32_t n_x;        /* particles per filter, 1..4096 (1..2048 for SMC2_AGE_SEIR)   */
    uint64_t seed;      /* Philox key of this run                                      */
    const int32_t* y;   /* host, T x n_obs row-major, non-negative (n_obs = 4 for AGE);
                           not read for SMC2_LINGAUSS                                   */
    const double* y_real; /* host, T finite reals: the observations of SMC2_LINGAUSS (not
                             read for the other models, may be NULL there)               */
} smc2_run;

/* Per-iteration record, SMC2_RECORD_LEN(D) doubles:
 *   [0] k   [1] ESS = l_k   [2] resampled (0/1)   [3] samples with zero weight
 *   [4] L-kernel fell back to the forward kernel (0/1)   [5] log sum_i w_k^i
 *   [6 .. 6+D)            posterior mean of theta at iteration k (Eq. realised_estimates)
 *   [6+D .. 6+D+D*D)      weighted covariance of theta
 *   [6+D+D*D .. 6+2D+D*D) weighted mean of the sampler coordinates phi
 *   [6+2D+D*D]            proposal used at iteration k (0 random walk, 1 learned,
 *                         2 Langevin, 3 population random walk)
 *   [7+2D+D*D]            learned proposal trained after iteration k: held-out mean
 *                         weighted NLL minus the random walk's (0 without training)    */
#define SMC2_RECORD_LEN(D) (8 + 2 * (D) + (D) * (D))

/* what smc2_dump copies (run r's slice, host_dst must hold the stated size) */
#define SMC2_DUMP_PHI 0      /* N x D  doubles: population after the last step            */
#define SMC2_DUMP_LP 1       /* N      doubles: its log-prior                              */
#define SMC2_DUMP_LL 2       /* N      doubles: its log-likelihood estimates               */
#define SMC2_DUMP_LOGW 3     /* N      doubles: its log-weights (0 after a resampling)     */
#define SMC2_DUMP_PHI_NEW 4  /* N x D  doubles: samples proposed in the last step          */
#define SMC2_DUMP_LP_NEW 5   /* N      doubles                                             */
#define SMC2_DUMP_LL_NEW 6   /* N      doubles: their particle-filter log-likelihoods      */
#define SMC2_DUMP_LOGW_PRE 7 /* N      doubles: log-weights before resampling              */
#define SMC2_DUMP_ANC 8      /* N      int32:   ancestors chosen (identity if no resampling) */
#define SMC2_DUMP_PSTEPS 15  /* 1      uint64:  particle-steps the run's filters executed since
                                smc2_init: N_x x the days each active filter ran (a filter
                                whose weights all vanish stops that day; inactive samples,
                                with zero weight or outside the prior's support, run none) */
#define SMC2_DUMP_THETA_NEW 17 /* N x D doubles: model parameters theta(phi_new) of the samples
                                  proposed in the last step (what their filters ran with)  */
#define SMC2_DUMP_SCORE 18     /* N x D doubles: the population's score estimates (natural
                                  parameters; SMC2_PROP_LANGEVIN only)                     */
#define SMC2_DUMP_SCORE_NEW 19 /* N x D doubles: the last step's proposals' score estimates */
#define SMC2_DUMP_LKFIT 16   /* 2D + 4D^2 doubles: moments of the last approximately optimal
                                L-kernel fit (Sec. IV-D), the weighted mean of the pairs
                                (phi_{k-1}, phi_k) then their weighted covariance (row-major,
                                2D x 2D); zero before the first fit */
/* learned proposal (SMC2_PROP_MLP only) */
#define SMC2_DUMP_MLP_OUT 9     /* N x P  float: network outputs at the population the
                                   last step proposed from (P = D + D(D+1)/2)            */
#define SMC2_DUMP_LOGQ 10       /* N      doubles: log q(phi_new | phi) of the learned
                                   proposal at the last step; 0 where that step drew from
                                   the prior (k = 1) or the random walk (also for the
                                   Langevin and population random-walk proposals: their
                                   log q at the last step)                                 */
#define SMC2_DUMP_MLP_PARAMS 11 /* NP     float: FP32 master weights W1[64][D] b1[64]
                                   W2[64][64] b2[64] W3[P][64] b3[P] (after training)    */
#define SMC2_DUMP_MLP_FRAME 12  /* D+D*D  doubles: input frame of the current network: the
                                   weighted mean c and the lower Cholesky factor F of the
                                   weighted covariance (row-major); inputs are F^-1(phi-c) */
#define SMC2_DUMP_MLP_STATE 13  /* 4      doubles: {use next iteration (0/1), Adam steps,
                                   held-out NLL of the network, of the random walk}      */
#define SMC2_DUMP_MLP_GRAD 14   /* NP     float: gradient of the last minibatch, before
                                   clipping, in the layout of SMC2_DUMP_MLP_PARAMS       */

/* One completed iteration of one run, as smc2_info reports it. The record's scalars
 * (Sec. IV: ESS = l_k before resampling, Eq. ess_smc2 and recycling_I; whether the
 * population was resampled, Eq. cdf and ncopies), the work the run's filters executed,
 * and the device time of the iteration's phases (all runs of the context together;
 * -1 where the iteration was replayed as one graph, whose phases are not timed). */
typedef struct {
    int32_t k;                /* iteration, 1-based                                          */
    int32_t resampled;        /* 1 when the population was resampled after the weights      */
    int32_t dead;             /* samples with zero weight                                    */
    int32_t lkernel_fallback; /* 1 when the Gaussian L-kernel fit was rejected              */
    int32_t learned;          /* 1 when the learned proposal drew the samples               */
    int32_t proposal;         /* the proposal that drew them: the record's column (0 random
                                 walk or prior draw, 1 learned, 2 Langevin, 3 population
                                 random walk)                                                */
    double ess;               /* effective sample size of the weights, = l_k                 */
    double log_weight_sum;    /* log sum_i w_k^i                                             */
    uint64_t particle_steps;  /* executed particle-steps of the run's filters (N_x x days
                                 each active filter ran)                                     */
    double ms_filters;        /* particle-filter launches                                    */
    double ms_outer;          /* proposal (prior draw / random walk / learned) and the outer
                                 update (L-kernel, weights, estimates, resampling)           */
    double ms_mlp;            /* learned proposal's network outputs and training (0 without) */
    double ms_step;           /* the whole iteration                                         */
} smc2_step_info;

/* Bytes of device workspace needed for this config and these runs (0 on bad input). */
size_t smc2_workspace_bytes(const smc2_config* cfg, int32_t n_runs, const smc2_run* runs);

/* Validate, copy the inputs to the workspace and prepare iteration k = 1.
 * hip_stream is a hipStream_t (NULL = the null stream). */
int smc2_init(const smc2_config* cfg, int32_t n_runs, const smc2_run* runs, void* d_workspace,
              size_t ws_bytes, void* hip_stream, smc2_ctx** out);

/* Enqueue iteration k = (number of previous steps) + 1 for every run. Returns
 * SMC2_E_STATE after K iterations. A run whose weights all vanish reports
 * SMC2_E_NUMERIC from the next synchronising call and keeps its previous population. */
int smc2_step(smc2_ctx* ctx);

/* Copy run `run`'s records of the completed iterations (k_done x SMC2_RECORD_LEN(D)
 * doubles) to host_dst; *k_done receives the number of completed iterations. */
int smc2_records(smc2_ctx* ctx, int32_t run, double* host_dst, size_t n_doubles, int32_t* k_done);

/* Information on completed iteration k (1 <= k <= iterations run) of run `run`.
 * Synchronises the stream. SMC2_E_ARG for a k that has not run. smc2_step itself returns
 * at once (the iteration runs asynchronously), so its information is read here. */
int smc2_info(smc2_ctx* ctx, int32_t run, int32_t k, smc2_step_info* info);

/* Posterior estimate of theta for run `run`: recycled over all completed iterations
 * with c_k = l_k / sum_j l_j (Sec. IV-C) when recycled != 0, else the last
 * iteration's. mean: D doubles; cov: D x D doubles or NULL. */
int smc2_estimate(smc2_ctx* ctx, int32_t run, int32_t recycled, double* mean, double* cov);

/* Copy one of the SMC2_DUMP_* arrays of run `run` to host memory (for tests). */
int smc2_dump(smc2_ctx* ctx, int32_t what, int32_t run, void* host_dst, size_t bytes);

/* Mean device time per iteration of the particle-filter kernels and of the whole
 * iteration, in milliseconds, over the steps since the last call (events on the
 * context's stream). Synchronises the stream. */
int smc2_timing(smc2_ctx* ctx, double* ms_pf, double* ms_step, int32_t* n_steps);

int smc2_destroy(smc2_ctx* ctx);

const char* smc2_last_error(const smc2_ctx* ctx);

/* The particle-filter launch groups of a context (filters sharing a workgroup size,
 * longest filters first) and the configuration each runs with. n_groups receives the
 * number of groups; for g < max_groups, desc[6g .. 6g+5] = {workgroup size, draw
 * schedule (SMC2_SCHED_PER_DRAW / SMC2_SCHED_POOLED), persistent (0/1), workgroups
 * launched, filters, dynamic LDS bytes per workgroup}, and tuned_ms[g] (may be NULL)
 * the time of the chosen configuration on the tuning sample (0 when not tuned).
 * Host-only; does not touch the device. */
int smc2_groups(const smc2_ctx* ctx, int32_t max_groups, int32_t* n_groups, int32_t* desc, float* tuned_ms);

/* ------------------------------------------------------------------ p-MCMC
 * Particle marginal Metropolis-Hastings (Sec. III, Eq. MHalgorithm_), the paper's
 * comparison method, on the same particle-filter kernels: `chains` independent chains,
 * each a Gaussian random walk on the sampler coordinates (covariance cfg->rw_cov) whose
 * target is the prior times the particle filter's likelihood estimate. The estimate of
 * the current state is kept until a proposal is accepted, so every chain targets the
 * exact posterior for any N_x (Andrieu, Doucet and Holenstein). The random walk is
 * symmetric, so the proposal densities of Eq. MHalgorithm_ cancel; a proposal outside
 * the prior's support is rejected without running its filter. Each chain starts from a
 * prior draw. Estimates are means over the chains' states after a burn-in.
 * Uses cfg's model, obs, D, precision, n_pop, prior, rw_cov, fixed, pf_always,
 * pf_resampling, block and schedule (N, K, proposal, lkernel, tune and the learned
 * proposal's settings are ignored). Random numbers (Philox, key = run->seed): chain c's
 * start from counter (c, 0, 0, 11<<24 | d), at iteration m its normals from
 * (c, 0, m<<16, 9<<24 | d) and its uniform from words 0 and 1 of (c, 0, m<<16, 10<<24);
 * its filter at iteration m runs as filter c of iteration m (0: the start).
 * Ownership, errors and synchronisation as for the sampler (smc2_last_error(NULL) gives
 * the message); smc2_pmcmc_step is asynchronous, the other calls synchronise. */
typedef struct smc2_pmcmc smc2_pmcmc;

#define SMC2_PMCMC_PHI 0         /* chains x (iterations+1) x D doubles: states (sampler coordinates),
                                    row 0 the start                                               */
#define SMC2_PMCMC_LL 1          /* chains x (iterations+1) doubles: their likelihood estimates    */
#define SMC2_PMCMC_LL_PROPOSED 2 /* chains x iterations doubles: the proposals' estimates (-inf
                                    outside the prior's support)                                  */
#define SMC2_PMCMC_ACCEPTED 3    /* chains x iterations int32: 1 where the proposal was accepted  */

/* Workspace bytes for `chains` chains (1..32768) of up to `iters` iterations (0..65535). */
size_t smc2_pmcmc_workspace_bytes(const smc2_config* cfg, int32_t chains, int32_t iters, const smc2_run* run);

/* Validate, copy the inputs and enqueue the chains' starts and their filters. */
int smc2_pmcmc_init(const smc2_config* cfg, int32_t chains, int32_t iters, const smc2_run* run, void* d_workspace,
                    size_t ws_bytes, void* hip_stream, smc2_pmcmc** out);

/* Enqueue n_iter further iterations of every chain; SMC2_E_STATE beyond `iters`. */
int smc2_pmcmc_step(smc2_pmcmc* ctx, int32_t n_iter);

/* Mean (D) and covariance (D x D, may be NULL) of theta over every chain's states after
 * the first burn_in iterations, and the acceptance rate over those iterations. */
int smc2_pmcmc_estimate(smc2_pmcmc* ctx, int32_t burn_in, double* mean, double* cov, double* accept_rate);

/* Copy one of the SMC2_PMCMC_* traces to host memory. */
int smc2_pmcmc_dump(smc2_pmcmc* ctx, int32_t what, void* host_dst, size_t bytes);

/* Device time of the iterations run by smc2_pmcmc_step (from the first step's start to
 * the last one's end) and the number of iterations run. */
int smc2_pmcmc_timing(smc2_pmcmc* ctx, double* ms, int32_t* iterations);

int smc2_pmcmc_destroy(smc2_pmcmc* ctx);

#ifdef __cplusplus
}
#endif
#endif
