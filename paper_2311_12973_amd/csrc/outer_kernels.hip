// outer_kernels.hip — the outer SMC^2 step (Sec. IV) in FP64 on gfx950.
//
// k_propose   one thread per sample: k = 1 draws from the prior (Eq. init_sample),
//             k > 1 moves with the Gaussian random walk (Eq. proposal); evaluates the
//             log-prior, the model parameters theta(phi) and whether the particle
//             filter has to run (a zero-weight sample or an out-of-support proposal
//             keeps weight zero and skips its filter).
// k_outer     one workgroup per run: approximately optimal Gaussian L-kernel fit and
//             conditioning (Sec. IV-D), weight update (Eq. l_weights), normalisation,
//             ESS = l_k (Eq. ess_smc2, recycling_I), estimates (Eq. realised_estimates),
//             integer systematic resampling (Eq. cdf, ncopies) as a prefix-sum search and
//             redistribution (Alg. 1) as a gather, reset (log w = 0), and the record.
// Moment sums over samples run sequentially in sample order, one thread per matrix
// entry, so they do not depend on the launch shape.
#include "block_ops.h"
#include "outer_kernels.h"

namespace smc2 {

#define LOG_2PI 1.8378770664093453

__device__ __forceinline__ double prior_logpdf(const OuterParams& p, const double* phi)
{
    double lp = 0.0;
    for (int d = 0; d < p.D; ++d) {
        const int fam = (int)p.prior[3 * d];
        const double a = p.prior[3 * d + 1], b = p.prior[3 * d + 2];
        if (fam == PRIOR_UNIFORM) {
            if (!(phi[d] >= a && phi[d] <= b)) return -INFINITY;
            lp += -log(b - a);
        } else {
            const double z = (phi[d] - a) / b;
            lp += (-0.5 * z * z - log(b)) - 0.5 * LOG_2PI;
        }
    }
    return lp;
}

__device__ __forceinline__ double theta_of(int fam, double v)
{
    if (fam == PRIOR_LOGNORMAL) return exp(v);
    if (fam == PRIOR_LOGITNORMAL) return 1.0 / (1.0 + exp(-v));
    return v;
}

__global__ void k_begin(int32_t* k_dev) { *k_dev += 1; }

__global__ void __launch_bounds__(256) k_propose(OuterArrays o, OuterParams p, const uint64_t* seeds)
{
    const int g = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (g >= p.R * p.N) return;
    const int D = p.D;
    const int r = g / p.N;
    const uint32_t i = (uint32_t)(g - r * p.N);
    const uint64_t seed = seeds[r];
    const uint32_t k = (uint32_t)(*o.k_dev);
    double phin[DMAX];
    if (k == 1) {
        for (int d = 0; d < D; ++d) {
            const W4 w = philox10(i, 0u, 1u << 16, (S_PRIOR << 24) | (uint32_t)d, (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
            const double u1 = u53(w.x, w.y), u2 = u53(w.z, w.w);
            const double a = p.prior[3 * d + 1], b = p.prior[3 * d + 2];
            if ((int)p.prior[3 * d] == PRIOR_UNIFORM) {
                phin[d] = a + (b - a) * u1;
            } else {
                const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
                phin[d] = a + b * z;
            }
        }
    } else {
        double z[DMAX];
        for (int d = 0; d < D; ++d) z[d] = normal_call(i, 0u, k << 16, (S_RW << 24) | (uint32_t)d, seed);
        const double* ph = o.phi + (size_t)g * D;
        for (int d = 0; d < D; ++d) {
            double acc = 0.0;
            for (int e = 0; e <= d; ++e) acc += p.lrw[d * D + e] * z[e];
            phin[d] = ph[d] + acc;
        }
    }
    const double lpn = prior_logpdf(p, phin);
    for (int d = 0; d < D; ++d) {
        o.phi_new[(size_t)g * D + d] = phin[d];
        o.theta_new[(size_t)g * D + d] = theta_of((int)p.prior[3 * d], phin[d]);
    }
    o.lp_new[g] = lpn;
    o.active[g] = (uint8_t)((k == 1) || (o.logw[g] != -INFINITY && lpn != -INFINITY));
}

// ---- small dense FP64 linear algebra (one thread) ----
__device__ int chol_lower(int n, const double* A, int lda, double* L)
{
    for (int a = 0; a < n * n; ++a) L[a] = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = A[j * lda + j];
        for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) return -1;
        L[j * n + j] = sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * lda + j];
            for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = v / L[j * n + j];
        }
    }
    return 0;
}

__device__ void chol_solve(int n, const double* L, double* b)
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

// log N(x; mu, L L^T)
__device__ double mvn_logpdf(int n, const double* x, const double* mu, const double* L, int ldl)
{
    double v[DMAX];
    double quad = 0.0, logdet = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = x[i] - mu[i];
        for (int k = 0; k < i; ++k) s -= L[i * ldl + k] * v[k];
        v[i] = s / L[i * ldl + i];
        quad += v[i] * v[i];
        logdet += log(L[i * ldl + i]);
    }
    return -0.5 * quad - logdet - 0.5 * n * LOG_2PI;
}

__global__ void __launch_bounds__(OUTER_BLOCK) k_outer(OuterArrays o, OuterParams p, const uint64_t* seeds)
{
    const int r = (int)blockIdx.x;
    const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
    const int N = p.N, D = p.D, D2 = 2 * D;
    const size_t base = (size_t)r * N;
    const uint32_t k = (uint32_t)(*o.k_dev);
    double* phi = o.phi + base * D;
    double* lp = o.lp + base;
    double* ll = o.ll + base;
    double* logw = o.logw + base;
    const double* phin = o.phi_new + base * D;
    const double* lpn = o.lp_new + base;
    const double* lln = o.ll_new + base;
    const double* thn = o.theta_new + base * D;
    double* lwp = o.logw_pre + base;
    double* wsc = o.scratch + base;
    uint64_t* qc = o.qc + base;
    int32_t* anc = o.anc + base;
    double* rec = o.records + ((size_t)r * p.K + (k - 1)) * p.rec_len;

    __shared__ RedLds red;
    __shared__ double mu[2 * DMAX], cov[4 * DMAX * DMAX], A[DMAX * DMAX], LS[DMAX * DMAX];
    __shared__ double mth[DMAX], mph[DMAX];
    __shared__ int fit_ok;

    // ---------------- approximately optimal L-kernel (k > 1)
    bool ratio_only = (p.lkernel == L_FORWARD);
    int fallback = 0;
    if (k >= 2 && p.lkernel == L_GAUSS_OPT) {
        double m0 = -INFINITY;
        for (int i = tid; i < N; i += nthr) m0 = logw[i] > m0 ? logw[i] : m0;
        const double M0 = block_max<double>(m0, &red);
        double s0 = 0.0;
        uint64_t z0 = 0, z1 = 0;
        for (int i = tid; i < N; i += nthr) s0 += exp(logw[i] - M0);
        block_sum3(s0, z0, z1, &red);
        const double W0 = M0 + log(s0);
        for (int i = tid; i < N; i += nthr) wsc[i] = exp(logw[i] - W0);
        __syncthreads();
        if (tid < D2) {
            double acc = 0.0;
            for (int i = 0; i < N; ++i) {
                const double z = tid < D ? phi[(size_t)i * D + tid] : phin[(size_t)i * D + tid - D];
                acc += wsc[i] * z;
            }
            mu[tid] = acc;
        }
        __syncthreads();
        if (tid < D2 * D2) {
            const int ea = tid / D2, ec = tid % D2;
            double acc = 0.0;
            for (int i = 0; i < N; ++i) {
                const double za = (ea < D ? phi[(size_t)i * D + ea] : phin[(size_t)i * D + ea - D]) - mu[ea];
                const double zc = (ec < D ? phi[(size_t)i * D + ec] : phin[(size_t)i * D + ec - D]) - mu[ec];
                acc += wsc[i] * za * zc;
            }
            cov[ea * D2 + ec] = acc;
        }
        __syncthreads();
        if (tid == 0) {
            double L22[DMAX * DMAX], S[DMAX * DMAX];
            int ok = chol_lower(D, cov + D * D2 + D, D2, L22) == 0;
            if (ok) {
                for (int rr = 0; rr < D; ++rr) {
                    double b[DMAX];
                    for (int c = 0; c < D; ++c) b[c] = cov[(D + c) * D2 + rr];
                    chol_solve(D, L22, b);
                    for (int c = 0; c < D; ++c) A[rr * D + c] = b[c];
                }
                for (int a2 = 0; a2 < D; ++a2)
                    for (int c = 0; c < D; ++c) {
                        double s = cov[a2 * D2 + c];
                        for (int e = 0; e < D; ++e) s -= A[a2 * D + e] * cov[(D + e) * D2 + c];
                        S[a2 * D + c] = s;
                    }
                ok = chol_lower(D, S, D, LS) == 0;
            }
            fit_ok = ok;
        }
        __syncthreads();
        if (!fit_ok) {
            ratio_only = true;
            fallback = 1;
        }
    }

    // ---------------- weight update
    uint64_t dead = 0;
    for (int i = tid; i < N; i += nthr) {
        double v;
        if (k == 1) {
            v = lln[i];
        } else {
            const double pin = lpn[i] + lln[i];
            if (logw[i] == -INFINITY || pin == -INFINITY) {
                v = -INFINITY;
            } else {
                v = (logw[i] + pin) - (lp[i] + ll[i]);
                if (!ratio_only) {
                    double m[DMAX];
                    for (int a2 = 0; a2 < D; ++a2) {
                        double s = mu[a2];
                        for (int c = 0; c < D; ++c) s += A[a2 * D + c] * (phin[(size_t)i * D + c] - mu[D + c]);
                        m[a2] = s;
                    }
                    const double lL = mvn_logpdf(D, phi + (size_t)i * D, m, LS, D);
                    const double lq = mvn_logpdf(D, phin + (size_t)i * D, phi + (size_t)i * D, p.lrw, D);
                    v = v + (lL - lq);
                }
            }
        }
        lwp[i] = v;
        dead += (v == -INFINITY);
    }
    double mloc = -INFINITY;
    for (int i = tid; i < N; i += nthr) mloc = lwp[i] > mloc ? lwp[i] : mloc;
    const double M = block_max<double>(mloc, &red);
    {
        double zz = 0.0;
        uint64_t z2 = 0;
        block_sum3(zz, dead, z2, &red);
    }
    if (M == -INFINITY) {
        for (int i = tid; i < N; i += nthr) {
            logw[i] = -INFINITY;
            anc[i] = i;
        }
        if (tid == 0) {
            for (int a2 = 0; a2 < p.rec_len; ++a2) rec[a2] = 0.0;
            rec[0] = (double)k;
            rec[3] = (double)dead;
            rec[4] = (double)fallback;
            rec[5] = -INFINITY;
            o.status[r] = -4;
        }
        return;
    }

    // ---------------- normalisation, quantised weights, ESS trigger
    double S = 0.0;
    uint64_t q1 = 0, q2 = 0;
    for (int i = tid; i < N; i += nthr) {
        const double w = exp(lwp[i] - M);
        S += w;
        const uint64_t q = (uint64_t)floor(w * 4294967296.0);
        qc[i] = q;
        const uint64_t h = q >> 8;
        q1 += h;
        q2 += h * h;
    }
    block_sum3(S, q1, q2, &red);
    const double W = M + log(S);
    double s2 = 0.0;
    for (int i = tid; i < N; i += nthr) {
        const double wn = exp(lwp[i] - W);
        wsc[i] = wn;
        s2 += wn * wn;
    }
    {
        uint64_t z1 = 0, z2 = 0;
        block_sum3(s2, z1, z2, &red);
    }
    const bool rs = ess_below_half(q1, q2, N);

    // ---------------- estimates at iteration k
    if (tid < D) {
        double acc = 0.0;
        for (int i = 0; i < N; ++i) acc += wsc[i] * thn[(size_t)i * D + tid];
        mth[tid] = acc;
    } else if (tid < D2) {
        double acc = 0.0;
        for (int i = 0; i < N; ++i) acc += wsc[i] * phin[(size_t)i * D + tid - D];
        mph[tid - D] = acc;
    }
    __syncthreads();
    if (tid < D * D) {
        const int ea = tid / D, ec = tid % D;
        double acc = 0.0;
        for (int i = 0; i < N; ++i)
            acc += wsc[i] * (thn[(size_t)i * D + ea] - mth[ea]) * (thn[(size_t)i * D + ec] - mth[ec]);
        rec[6 + D + tid] = acc;
    }
    if (tid == 0) {
        rec[0] = (double)k;
        rec[1] = 1.0 / s2;
        rec[2] = rs ? 1.0 : 0.0;
        rec[3] = (double)dead;
        rec[4] = (double)fallback;
        rec[5] = W;
        for (int a2 = 0; a2 < D; ++a2) {
            rec[6 + a2] = mth[a2];
            rec[6 + D + D * D + a2] = mph[a2];
        }
        o.status[r] = 0;
    }

    // ---------------- resampling (Sec. IV-B) and redistribution
    if (rs) {
        __syncthreads();
        const uint64_t Q = block_scan_lds(qc, N, &red);
        const W4 wd = philox10(0u, 0u, k << 16, S_OUTER_RS << 24, (uint32_t)seeds[r], (uint32_t)(seeds[r] >> 32));
        block_ancestors(qc, N, Q, (uint64_t)wd.x | ((uint64_t)wd.y << 32), anc);
    } else {
        for (int i = tid; i < N; i += nthr) anc[i] = i;
    }
    __syncthreads();
    for (int m = tid; m < N; m += nthr) {
        const int s = anc[m];
        for (int d = 0; d < D; ++d) phi[(size_t)m * D + d] = phin[(size_t)s * D + d];
        lp[m] = lpn[s];
        ll[m] = lln[s];
        logw[m] = rs ? 0.0 : lwp[m];
    }
}

hipError_t launch_begin_iteration(const OuterArrays& o, hipStream_t s)
{
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(1), 0, s, o.k_dev);
    return hipGetLastError();
}

hipError_t launch_propose(const OuterArrays& o, const OuterParams& p, const uint64_t* d_seeds, hipStream_t s)
{
    const int total = p.R * p.N;
    hipLaunchKernelGGL(k_propose, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, o, p, d_seeds);
    return hipGetLastError();
}

hipError_t launch_outer_update(const OuterArrays& o, const OuterParams& p, const uint64_t* d_seeds,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_outer, dim3((unsigned)p.R), dim3(OUTER_BLOCK), 0, s, o, p, d_seeds);
    return hipGetLastError();
}

}  // namespace smc2
