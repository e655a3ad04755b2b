/*
 * smc2_kernels.h — kernel-level entry points of libsmc2.so.
 *
 * They run single building blocks of the sampler on device arrays so that each can
 * be compared element by element with an independent implementation; the sampler
 * itself (smc2.h) uses the same device code. All pointers prefixed d_ are device
 * memory owned by the caller; nothing is allocated. Calls are asynchronous on the
 * given HIP stream (NULL = null stream). Return SMC2_OK or a negative SMC2_E_* code
 * (see smc2.h); smc2_last_error(NULL) describes the last failure of the thread.
 */
#ifndef SMC2_KERNELS_H
#define SMC2_KERNELS_H

#include <stddef.h>
#include <stdint.h>

#include "smc2.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 block function (Salmon et al., SC'11): d_out[4e..4e+3] = Philox(counter
 * d_ctr[4e..4e+3], key = (seed low word, seed high word)) for e < n. */
int smc2_philox_batch(int32_t n, const uint32_t* d_ctr, uint64_t seed, uint32_t* d_out, void* hip_stream);

/* Binomial(d_n[j], d_p[j]) draws of the particle-filter sampler (the flows of the
 * chain-binomial model, Sec. V-A) at coordinates (particle j, filter i, iteration k,
 * day t, draw b), j < count, in precision SMC2_PREC_FP32 (d_p rounded to FP32) or
 * SMC2_PREC_FP64. d_n: int32[count], each below 2^30 (n <= 0 draws 0); d_p:
 * double[count]; d_out: int32[count]. */
int smc2_binomial_batch(int32_t precision, int32_t count, const int32_t* d_n, const double* d_p, uint64_t seed,
                        uint32_t i, uint32_t k, uint32_t t, uint32_t b, int32_t* d_out, void* hip_stream);

/* Integer systematic resampling (Sec. IV-B, Eq. cdf and ncopies, Alg. 1) of n_sets
 * independent sets of n quantised weights (d_q: uint64[n_sets][n], each set with a
 * positive total below 2^47): d_anc[s][m] = min{ j : n C_j > m Q + U } with C the
 * inclusive cumulative sum, Q the total and U = floor(d_x64[s] Q / 2^64);
 * d_trigger[s] = 1 when ESS < n/2 on q >> 8 (exact integer test). 1 <= n <= 4096. */
int smc2_resample_batch(int32_t n_sets, int32_t n, const uint64_t* d_q, const uint64_t* d_x64, int32_t* d_anc,
                        int32_t* d_trigger, void* hip_stream);

/* Device workspace bytes for smc2_pf_loglik (and the other filter entry points): the
 * staged run and observations. A size only: the entry points validate the rest of cfg
 * and run when called. 0 (with a message) when cfg or run is NULL or run->T < 1. */
size_t smc2_pf_workspace_bytes(const smc2_config* cfg, const smc2_run* run);

/* Particle-filter log-likelihood estimates (Sec. II) for n_theta model parameter
 * vectors d_theta (double[n_theta][D], natural parameters, not sampler coordinates)
 * on the observations of `run`: filter index i = row of d_theta, iteration index k
 * (selects the random streams). d_ll: double[n_theta]. Uses cfg's model, obs,
 * precision, pf_always, n_pop, fixed and block; N, K, prior and proposal are ignored. */
int smc2_pf_loglik(const smc2_config* cfg, int32_t n_theta, const double* d_theta, const smc2_run* run,
                   uint32_t k, double* d_ll, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* smc2_pf_loglik without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid allocation): the
 * run descriptor and the observation series are staged in a static device array of
 * the library (16640 bytes per device, held until the process ends) instead of
 * d_workspace. The array covers every valid run (T <= 1024, up to 4 observation series);
 * a run needing more is rejected with SMC2_E_ARG. Nothing is allocated: no hipMalloc,
 * hipFree or allocating library call. Results are identical to smc2_pf_loglik's. Like
 * smc2_pf_loglik the call returns after the stream has run the filters. Every call on
 * one device shares that device's array: calls that overlap on one device (from
 * several threads, or on several streams) race and must be serialised by the caller. */
int smc2_pf_loglik_noalloc(const smc2_config* cfg, int32_t n_theta, const double* d_theta, const smc2_run* run,
                           uint32_t k, double* d_ll, void* hip_stream);

/* As smc2_pf_loglik, and also writes every filter's per-day log-likelihood
 * increments (d_inc: double[n_theta][T]) and resampling flags (d_rs:
 * int32[n_theta][T]); a filter that dies at day t records -inf at t and 0 after. */
int smc2_pf_trace(const smc2_config* cfg, int32_t n_theta, const double* d_theta, const smc2_run* run, uint32_t k,
                  double* d_ll, double* d_inc, int32_t* d_rs, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* As smc2_pf_trace, and also writes every filter's particle counts of each day
 * before resampling (d_state: int32[n_theta][T][n_counts][n_x], n_counts = 2 / 3 / 12
 * for SIR / SEIR / age-structured SEIR; for SMC2_LINGAUSS n_counts = 2, the low and
 * high 32-bit words of each particle's FP64 state) and, when d_anc is not NULL, the ancestors
 * chosen after each day (d_anc: int32[n_theta][T][n_x]; the identity on days without
 * resampling; rows after a filter's death day are left unwritten). Together with d_rs
 * these are the filter's integer decisions, from which an FP64 replay of Sec. II's
 * weights recomputes its likelihood estimate. */
int smc2_pf_trace_state(const smc2_config* cfg, int32_t n_theta, const double* d_theta, const smc2_run* run,
                        uint32_t k, double* d_ll, double* d_inc, int32_t* d_rs, int32_t* d_state, int32_t* d_anc,
                        void* d_workspace, size_t ws_bytes, void* hip_stream);

/* Score of the log-likelihood estimate (the gradient of log p(y | theta) on the natural
 * parameters; by Fisher's identity the posterior mean of the complete-data score, Sec. II
 * filter): each particle carries its trajectory's running score (per flow
 * d log Bin / d theta through the hazard, d log NB / d r when r is a parameter; for
 * SMC2_LINGAUSS the derivatives of the two Gaussian densities), resampling moves it with
 * the particle, and the last day's weights average it. The estimate is consistent in
 * n_x, not unbiased. d_ll: double[n_theta], the same estimates as smc2_pf_loglik's;
 * d_score: double[n_theta][D]. SIR (D = 2), SEIR (D = 4 or 5; the initial fraction iota
 * enters only through a rounding and gets 0) and SMC2_LINGAUSS (D = 3, needs
 * sigma_x > 0); other models return SMC2_E_UNSUPPORTED. A filter whose weights all
 * vanish gets -inf and a zero score. The scores sit in LDS beside the counts. Draw
 * schedule: per draw (SMC2_SCHED_AUTO or SMC2_SCHED_PER_DRAW; n_x up to 2048, for SEIR
 * in FP64 with T <= 365) or pooled (SMC2_SCHED_POOLED, SIR and SEIR, n_x up to about
 * 1024 with the scores; faster only for small filters), the same bits either way. A
 * schedule that does not fit returns SMC2_E_ARG. The workspace is
 * smc2_pf_workspace_bytes'. Returns after the stream has run the filters. */
int smc2_pf_score(const smc2_config* cfg, int32_t n_theta, const double* d_theta, const smc2_run* run, uint32_t k,
                  double* d_ll, double* d_score, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* Learned proposal, network outputs (SMC2_PROP_MLP). d_params: FP32 weights in the
 * layout of SMC2_DUMP_MLP_PARAMS for dimension D (1..8); d_frame: D + D*D doubles
 * (mean c, lower Cholesky factor F row-major; the inputs are F^-1 (phi - c)); d_phi:
 * n x D doubles (sampler coordinates); d_out: n x P floats, P = D +
 * D(D+1)/2, the outputs a (mean) and the packed Cholesky entries before the softplus
 * of the diagonal. Matrix products take BF16-rounded operands with FP32 accumulation.
 * All pointers are device memory owned by the caller. Asynchronous on the stream;
 * SMC2_E_ARG on bad sizes or null pointers. */
int smc2_mlp_forward(int32_t D, int32_t n, const float* d_params, const double* d_frame, const double* d_phi,
                     float* d_out, void* hip_stream);

/* Learned proposal, gradient of one minibatch: d_grad (NP floats) receives the
 * parameter gradient and d_loss (1 double) the value of sum_r w_r NLL(u_t,r | u_in,r)
 * over the n rows (inputs d_phi_in, targets d_phi_t, n x D doubles; row weights d_w,
 * n doubles), as the training step computes it (no clipping, no update). n <= 32768. */
int smc2_mlp_grad(int32_t D, int32_t n, const float* d_params, const double* d_frame, const double* d_phi_in,
                  const double* d_phi_t, const double* d_w, float* d_grad, double* d_loss, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
