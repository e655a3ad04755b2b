// pmcmc_kernels.h — launch interface of the particle marginal Metropolis-Hastings
// kernels (Sec. III, the paper's comparison method): C independent chains advance
// together, one proposal, one filter launch over all chains and one decision per
// iteration.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc2 {

struct McArrays {
    double* phi;        // [C][D] current states (sampler coordinates)
    double* lp;         // [C]    their log-prior
    double* ll;         // [C]    their likelihood estimates (kept until a proposal is accepted)
    double* phi_new;    // [C][D] proposals
    double* theta_new;  // [C][D] model parameters of the proposals (the filters' input)
    double* lp_new;     // [C]
    double* ll_new;     // [C]    the filters' output
    uint8_t* active;    // [C]    1: the proposal lies in the prior's support, run its filter
    double* phi_trace;  // [C][iters + 1][D] states after each iteration (0: the start)
    double* ll_trace;   // [C][iters + 1]
    double* lln_trace;  // [C][iters] the proposals' estimates (-inf outside the support)
    int32_t* acc_trace; // [C][iters] 1: accepted
    int32_t* m_dev;     // iteration counter (0: the start)
};

struct McParams {
    int32_t C, D, iters;
    const double* prior;  // [D][3] {family, a, b} (device)
    const double* lrw;    // [D][D] lower Cholesky factor of the random-walk covariance (device)
};

// chains' starting points (prior draws) as proposals of iteration 0
hipError_t launch_mc_start(const McArrays& a, const McParams& p, uint64_t seed, hipStream_t s);
// advance the iteration counter, then the random-walk proposals of every chain
hipError_t launch_mc_propose(const McArrays& a, const McParams& p, uint64_t seed, hipStream_t s);
// the Metropolis-Hastings decisions (iteration 0: take the starting points) and traces
hipError_t launch_mc_accept(const McArrays& a, const McParams& p, uint64_t seed, hipStream_t s);

}  // namespace smc2
