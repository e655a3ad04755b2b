// pmcmc_kernels.hip — particle marginal Metropolis-Hastings (Sec. III, Eq. MHalgorithm_)
// on gfx950, one thread per chain; the chains' filters run in the particle-filter batch
// kernel between the proposal and the decision.
//
// A chain moves by a Gaussian random walk on the sampler coordinates (the covariance of
// the configuration). The target density is the prior times the filter's likelihood
// estimate, and the estimate of the current state is kept until a proposal is accepted
// (it travels with the state): the chain then targets the exact posterior for any number
// of particles. The random walk is symmetric, so the proposal densities of Eq.
// MHalgorithm_ cancel. A proposal outside the prior's support is rejected without a filter.
// Random numbers (Philox, key = the seed), chain c: starting point coordinate d from
// (c, 0, 0, 11<<24 | d) like the sampler's prior draw; at iteration m the normal of
// coordinate d from (c, 0, m<<16, 9<<24 | d) and the uniform from words 0, 1 of
// (c, 0, m<<16, 10<<24); the filter of chain c at iteration m: filter c, iteration m.
#include "block_ops.h"
#include "outer_kernels.h"
#include "pmcmc_kernels.h"

namespace smc2 {

enum : uint32_t { S_MCMC_RW = 9u, S_MCMC_U = 10u, S_MCMC_INIT = 11u };

__global__ void k_mc_begin(int32_t* m_dev)
{
    if (threadIdx.x == 0) *m_dev += 1;
}

template <int D>
__global__ void __launch_bounds__(256) k_mc_start(McArrays a, McParams p, uint64_t seed)
{
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= p.C) return;
    double phi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const W4 w = philox10((uint32_t)c, 0u, 0u, (S_MCMC_INIT << 24) | (uint32_t)d, (uint32_t)seed,
                              (uint32_t)(seed >> 32));
        const double u1 = u53(w.x, w.y), u2 = u53(w.z, w.w);
        const double lo = p.prior[3 * d + 1], hi = p.prior[3 * d + 2];
        if ((int)p.prior[3 * d] == PRIOR_UNIFORM) phi[d] = lo + (hi - lo) * u1;
        else phi[d] = lo + hi * (sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
    }
    const double lp = prior_logpdf<D>(p.prior, phi);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        a.phi_new[(size_t)c * D + d] = phi[d];
        a.theta_new[(size_t)c * D + d] = theta_of((int)p.prior[3 * d], phi[d]);
    }
    a.lp_new[c] = lp;
    a.active[c] = (uint8_t)(lp != -INFINITY);
}

template <int D>
__global__ void __launch_bounds__(256) k_mc_propose(McArrays a, McParams p, uint64_t seed)
{
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= p.C) return;
    const uint32_t m = (uint32_t)(*a.m_dev);
    double z[D], phn[D];
#pragma unroll
    for (int d = 0; d < D; ++d) z[d] = normal_call((uint32_t)c, 0u, m << 16, (S_MCMC_RW << 24) | (uint32_t)d, seed);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e <= d; ++e) acc += p.lrw[d * D + e] * z[e];
        phn[d] = a.phi[(size_t)c * D + d] + acc;
    }
    const double lp = prior_logpdf<D>(p.prior, phn);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        a.phi_new[(size_t)c * D + d] = phn[d];
        a.theta_new[(size_t)c * D + d] = theta_of((int)p.prior[3 * d], phn[d]);
    }
    a.lp_new[c] = lp;
    a.active[c] = (uint8_t)(lp != -INFINITY);
}

// Eq. MHalgorithm_ with a symmetric proposal: accept when the proposal has positive
// target and either the current state has none or log u < its log-target ratio
__device__ __forceinline__ bool mh_accept(double lp, double ll, double lp_new, double ll_new, double u)
{
    const double cur = lp + ll, nw = lp_new + ll_new;
    if (nw == -INFINITY) return false;
    if (cur == -INFINITY) return true;
    return log(u) < nw - cur;
}

template <int D>
__global__ void __launch_bounds__(256) k_mc_accept(McArrays a, McParams p, uint64_t seed)
{
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= p.C) return;
    const int m = *a.m_dev;
    const double lln = a.active[c] ? a.ll_new[c] : -INFINITY;
    bool take = m == 0;
    if (m > 0) {
        const W4 w = philox10((uint32_t)c, 0u, (uint32_t)m << 16, S_MCMC_U << 24, (uint32_t)seed, (uint32_t)(seed >> 32));
        take = mh_accept(a.lp[c], a.ll[c], a.lp_new[c], lln, u53(w.x, w.y));
        a.lln_trace[(size_t)c * p.iters + (m - 1)] = lln;
        a.acc_trace[(size_t)c * p.iters + (m - 1)] = take ? 1 : 0;
    }
    if (take) {
#pragma unroll
        for (int d = 0; d < D; ++d) a.phi[(size_t)c * D + d] = a.phi_new[(size_t)c * D + d];
        a.lp[c] = a.lp_new[c];
        a.ll[c] = lln;
    }
    const size_t row = (size_t)c * (p.iters + 1) + m;
#pragma unroll
    for (int d = 0; d < D; ++d) a.phi_trace[row * D + d] = a.phi[(size_t)c * D + d];
    a.ll_trace[row] = a.ll[c];
}

namespace {
template <int D> hipError_t launch_d(int which, const McArrays& a, const McParams& p, uint64_t seed, hipStream_t s)
{
    const dim3 grid((unsigned)((p.C + 255) / 256)), blk(256);
    if (which == 0) hipLaunchKernelGGL(k_mc_start<D>, grid, blk, 0, s, a, p, seed);
    if (which == 1) {
        hipLaunchKernelGGL(k_mc_begin, dim3(1), dim3(64), 0, s, a.m_dev);
        hipLaunchKernelGGL(k_mc_propose<D>, grid, blk, 0, s, a, p, seed);
    }
    if (which == 2) hipLaunchKernelGGL(k_mc_accept<D>, grid, blk, 0, s, a, p, seed);
    return hipGetLastError();
}

hipError_t dispatch(int which, const McArrays& a, const McParams& p, uint64_t seed, hipStream_t s)
{
    switch (p.D) {
    case 1: return launch_d<1>(which, a, p, seed, s);
    case 2: return launch_d<2>(which, a, p, seed, s);
    case 3: return launch_d<3>(which, a, p, seed, s);
    case 4: return launch_d<4>(which, a, p, seed, s);
    case 5: return launch_d<5>(which, a, p, seed, s);
    case 6: return launch_d<6>(which, a, p, seed, s);
    case 7: return launch_d<7>(which, a, p, seed, s);
    case 8: return launch_d<8>(which, a, p, seed, s);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_mc_start(const McArrays& a, const McParams& p, uint64_t seed, hipStream_t s)
{
    return dispatch(0, a, p, seed, s);
}
hipError_t launch_mc_propose(const McArrays& a, const McParams& p, uint64_t seed, hipStream_t s)
{
    return dispatch(1, a, p, seed, s);
}
hipError_t launch_mc_accept(const McArrays& a, const McParams& p, uint64_t seed, hipStream_t s)
{
    return dispatch(2, a, p, seed, s);
}

}  // namespace smc2
