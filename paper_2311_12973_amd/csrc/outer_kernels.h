// outer_kernels.h — launch interface of the outer SMC^2 step (FP64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc2 {

enum : int { PRIOR_UNIFORM = 0, PRIOR_LOGNORMAL = 1, PRIOR_LOGITNORMAL = 2, PRIOR_NORMAL = 3 };
enum : int { L_FORWARD = 0, L_GAUSS_OPT = 1 };
constexpr int OUTER_BLOCK = 256;
constexpr int DMAX = 8;

// Per-run device arrays of the outer sampler (each run holds N samples).
struct OuterArrays {
    double* phi;       // [R][N][D] current population (sampler coordinates)
    double* lp;        // [R][N]    its log-prior
    double* ll;        // [R][N]    its log-likelihood estimate
    double* logw;      // [R][N]    its log-weight
    double* phi_new;   // [R][N][D] proposals of this iteration
    double* lp_new;    // [R][N]
    double* ll_new;    // [R][N]    particle-filter output
    double* theta_new; // [R][N][D] model parameters of the proposals
    double* logw_pre;  // [R][N]    weights before resampling
    double* scratch;   // [R][N]    normalised weights
    uint64_t* qc;      // [R][N]    quantised weights / cumulative sums
    int32_t* anc;      // [R][N]
    uint8_t* active;   // [R][N]    run the particle filter for this proposal
    double* records;   // [R][K][record_len]
    int32_t* status;   // [R]       0, or -4 when every weight of the run vanished
    double* lkfit;     // [R][2D + 4D^2] moments of the last L-kernel fit: mean of (phi_{k-1},
                       //               phi_k), then its weighted covariance (row-major)
    int32_t* k_dev;    // iteration counter
    const unsigned long long* psteps;  // [R]    executed particle-steps so far (filter kernel)
    unsigned long long* psteps_at;     // [R][K] its value after each iteration's filters
    // learned proposal (NULL unless the configuration uses it)
    const int32_t* mlp_use;   // [R]        1: this iteration proposes with the network
    const float* mlp_out;     // [R][N][P]  network outputs at the current population
    const double* mlp_frame;  // [R][D+D*D] input frame of the network: mean c, Cholesky factor F
    double* logq;             // [R][N]     log q(phi_new | phi) of the learned proposal or of a
                              //            proposal with the population's covariance
    // Langevin proposal (NULL unless configured): score estimates on the natural parameters
    double* score;            // [R][N][D]  of the population (they travel with their samples)
    double* score_new;        // [R][N][D]  of the proposals (the filters' output)
    double* pop_chol;         // [R][D][D]  Cholesky factor of the proposing population's
                              //            weighted covariance (the proposal covariance of the
                              //            Langevin and population random-walk proposals)
};

struct OuterParams {
    int32_t N, D, K, R;
    int32_t lkernel;
    int32_t rec_len;
    const double* prior; // [D][3] {family, a, b} (device)
    const double* lrw;   // [D][D] lower Cholesky factor of the RW covariance (device)
    int32_t mlp;         // 1: the learned proposal is configured
    int32_t langevin;    // 1: the truncated Langevin proposal is configured (drift + scores)
    int32_t popcov;      // 1: the proposal covariance is the proposing population's (the
                         //    Langevin proposal and the population random walk)
    double lgv_step;     // Langevin proposal: the fraction of the truncated drift applied
};

// model parameter theta_d from the sampler coordinate phi_d of a prior family
__device__ __forceinline__ double theta_of(int fam, double v)
{
    if (fam == PRIOR_LOGNORMAL) return exp(v);
    if (fam == PRIOR_LOGITNORMAL) return 1.0 / (1.0 + exp(-v));
    return v;
}

// log prior density on the sampler coordinates (prior: D x {family, a, b}); -inf outside
// a uniform prior's support
template <int D> __device__ __forceinline__ double prior_logpdf(const double* prior, const double* phi)
{
    double lp = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int fam = (int)prior[3 * d];
        const double a = prior[3 * d + 1], b = prior[3 * d + 2];
        if (fam == PRIOR_UNIFORM) {
            lp = (phi[d] >= a && phi[d] <= b && lp != -INFINITY) ? lp + -log(b - a) : -INFINITY;
        } else {
            const double zz = (phi[d] - a) / b;
            lp = lp + ((-0.5 * zz * zz - log(b)) - 0.5 * 1.8378770664093453);
        }
    }
    return lp;
}

hipError_t launch_begin_iteration(const OuterArrays& o, int32_t* queues, int n_queues, hipStream_t s);
hipError_t launch_propose(const OuterArrays& o, const OuterParams& p, const uint64_t* d_seeds, hipStream_t s);
// Langevin and population random-walk proposals: the proposing population's weighted
// covariance factor (k > 1)
hipError_t launch_pop_frame(const OuterArrays& o, const OuterParams& p, hipStream_t s);
hipError_t launch_outer_update(const OuterArrays& o, const OuterParams& p, const uint64_t* d_seeds,
                               hipStream_t s);

}  // namespace smc2
