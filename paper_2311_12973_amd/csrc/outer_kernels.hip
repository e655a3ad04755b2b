// outer_kernels.hip — the outer SMC^2 step (Sec. IV) in FP64 on gfx950.
//
// k_propose   one thread per sample: k = 1 draws from the prior (Eq. init_sample),
//             k > 1 moves with the Gaussian random walk (Eq. proposal); evaluates the
//             log-prior, the model parameters theta(phi) and whether the particle
//             filter has to run (a zero-weight sample or an out-of-support proposal
//             keeps weight zero and skips its filter).
// k_outer     one workgroup per run: approximately optimal Gaussian L-kernel fit and
//             conditioning (Sec. IV-D; without a usable fit, the random walk's Gaussian
//             read backwards), weight update (Eq. l_weights), normalisation,
//             ESS = l_k (Eq. ess_smc2, recycling_I), estimates (Eq. realised_estimates),
//             integer systematic resampling (Eq. cdf, ncopies) as a prefix-sum search and
//             redistribution (Alg. 1) as a gather, reset (log w = 0), and the record.
// k_propose and k_outer are instantiated per parameter dimension D (1..8), so the
// per-sample vectors live in registers. Moment sums over samples are workgroup
// reductions in a fixed order (a fixed 256-thread workgroup), so the result does not
// depend on anything but N.
#include "block_ops.h"
#include "outer_kernels.h"

namespace smc2 {

#define LOG_2PI 1.8378770664093453
// relative numerical-rank floor of the L-kernel fit
#define LK_REL_FLOOR 1e-12

// Advances the device iteration counter and zeroes the particle filter's work-list
// counters (a kernel, so that a captured iteration holds no memset node).
__global__ void k_begin(int32_t* k_dev, int32_t* queues, int n_queues)
{
    if (threadIdx.x == 0) *k_dev += 1;
    for (int i = (int)threadIdx.x; i < n_queues; i += (int)blockDim.x) queues[i] = 0;
}

template <int D> __device__ __forceinline__ double mvn_logpdf(const double* x, const double* mu, const double* L);

template <int D>
__global__ void __launch_bounds__(256) k_propose(OuterArrays o, OuterParams p, const uint64_t* seeds)
{
    const int g = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (g >= p.R * p.N) return;
    const int r = g / p.N;
    const uint32_t i = (uint32_t)(g - r * p.N);
    const uint64_t seed = seeds[r];
    const uint32_t k = (uint32_t)(*o.k_dev);
    double phin[D];
    if (k == 1) {
#pragma unroll
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
        double z[D];
#pragma unroll
        for (int d = 0; d < D; ++d) z[d] = normal_call(i, 0u, k << 16, (S_RW << 24) | (uint32_t)d, seed);
        if (p.mlp && o.mlp_use[r]) {
            // learned proposal: phi' = c + F (a + L z) from the network outputs at phi,
            // with its exact log-density (normalisation Jacobian included)
            constexpr int P = D + D * (D + 1) / 2;
            const float* out = o.mlp_out + (size_t)g * P;
            const double* fr = o.mlp_frame + (size_t)r * (D + D * D);
            double L[D * (D + 1) / 2];
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b) {
                    const double x = (double)out[D + a * (a + 1) / 2 + b];
                    L[a * (a + 1) / 2 + b] = (a == b) ? (x > 30.0 ? x : log1p(exp(x))) + 1e-3 : x;
                }
            double lq = -0.5 * D * LOG_2PI, u[D];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                double sa = (double)out[a];
#pragma unroll
                for (int b = 0; b <= a; ++b) sa += L[a * (a + 1) / 2 + b] * z[b];
                u[a] = sa;
                lq -= 0.5 * z[a] * z[a] + log(L[a * (a + 1) / 2 + a]) + log(fr[D + a * D + a]);
            }
#pragma unroll
            for (int a = 0; a < D; ++a) {
                double sa = fr[a];
#pragma unroll
                for (int b = 0; b <= a; ++b) sa += fr[D + a * D + b] * u[b];
                phin[a] = sa;
            }
            o.logq[g] = lq;
        } else if (p.popcov) {
            // Sigma = L L' the weighted covariance of the proposing population; phi' = m + L z.
            // The population random walk: m = phi. The truncated Langevin proposal:
            // m = phi + delta, delta = s times 1/2 Sigma g shrunk to Mahalanobis length 1, g
            // the gradient of log(prior x likelihood) on the sampler coordinates from the
            // score estimate that travelled with the sample, s the step fraction.
            const double* ph = o.phi + (size_t)g * D;
            const double* Lq = o.pop_chol + (size_t)r * D * D;
            double m[D];
#pragma unroll
            for (int d = 0; d < D; ++d) m[d] = ph[d];
            if (p.langevin) {
                const double* sth = o.score + (size_t)g * D;
                double gr[D], v[D];
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int fam = (int)p.prior[3 * d];
                    const double a = p.prior[3 * d + 1], b = p.prior[3 * d + 2];
                    const double th = theta_of(fam, ph[d]);
                    const double J =
                        fam == PRIOR_LOGNORMAL ? th : (fam == PRIOR_LOGITNORMAL ? th * (1.0 - th) : 1.0);
                    const double gp = fam == PRIOR_UNIFORM ? 0.0 : -(ph[d] - a) / (b * b);
                    gr[d] = J * sth[d] + gp;
                }
                double n2 = 0.0;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    double acc = 0.0;
#pragma unroll
                    for (int c = a; c < D; ++c) acc += Lq[c * D + a] * gr[c];
                    v[a] = acc;
                    n2 += acc * acc;
                }
                const double len = 0.5 * sqrt(n2);
                const double shrink = len > 1.0 ? 1.0 / len : 1.0;
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    double acc = 0.0;
#pragma unroll
                    for (int c = 0; c <= a; ++c) acc += Lq[a * D + c] * v[c];
                    m[a] = ph[a] + p.lgv_step * ((0.5 * acc) * shrink);
                }
            }
#pragma unroll
            for (int a = 0; a < D; ++a) {
                double lz = 0.0;
#pragma unroll
                for (int c = 0; c <= a; ++c) lz += Lq[a * D + c] * z[c];
                phin[a] = m[a] + lz;
            }
            o.logq[g] = mvn_logpdf<D>(phin, m, Lq);
        } else {
            const double* ph = o.phi + (size_t)g * D;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                double acc = 0.0;
#pragma unroll
                for (int e = 0; e <= d; ++e) acc += p.lrw[d * D + e] * z[e];
                phin[d] = ph[d] + acc;
            }
        }
    }
    // the learned proposal's density is stored where it proposed; 0 marks the other draws
    if (p.mlp && (k == 1 || !o.mlp_use[r])) o.logq[g] = 0.0;
    const double lpn = prior_logpdf<D>(p.prior, phin);
#pragma unroll
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

// log N(x; mu, L L^T), L row-major D x D
template <int D> __device__ __forceinline__ double mvn_logpdf(const double* x, const double* mu, const double* L)
{
    double v[D];
    double quad = 0.0, logdet = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s = x[i] - mu[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i * D + k] * v[k];
        v[i] = s / L[i * D + i];
        quad += v[i] * v[i];
        logdet += log(L[i * D + i]);
    }
    return -0.5 * quad - logdet - 0.5 * D * LOG_2PI;
}

constexpr int OUTER_WAVES = OUTER_BLOCK / 64;
constexpr int VSUM_MAX = 18;  // widest block_sum_vec (2 D + 1 = 17 for D = 8; covariance passes up to 18)

// Sum of E per-thread values over the block, in a fixed order (butterfly inside each
// wave, then the waves in index order); every thread then reads the E sums from out[]
// (LDS). lds holds OUTER_WAVES x E doubles.
template <int E>
__device__ __forceinline__ void block_sum_vec(double (&v)[E], double* lds, double* out)
{
    static_assert(E <= VSUM_MAX, "block_sum_vec width");
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = wave_sum(v[e]);
    if (lane_id() == 0)
#pragma unroll
        for (int e = 0; e < E; ++e) lds[wave_id() * E + e] = v[e];
    __syncthreads();
    if ((int)threadIdx.x < E) {
        double s = 0.0;
        for (int w = 0; w < OUTER_WAVES; ++w) s += lds[w * E + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// out (NV x NV, symmetric) = sum_i w_i (z_i - m)(z_i - m)^T, z_i loaded by load(i, z).
// The NV (NV + 1) / 2 upper-triangle entries are accumulated in as few passes as the
// reduction width allows (at most VSUM_MAX partial sums per thread), each pass ending
// in one block reduction. Every entry is summed in the same order however the entries
// are grouped into passes.
// row and column of each upper-triangle entry of an NV x NV matrix, row by row
template <int NV> struct TriIndex {
    int row[NV * (NV + 1) / 2], col[NV * (NV + 1) / 2];
    constexpr TriIndex() : row(), col()
    {
        int e = 0;
        for (int a = 0; a < NV; ++a)
            for (int c = a; c < NV; ++c) {
                row[e] = a;
                col[e] = c;
                ++e;
            }
    }
};

template <int NV, class Load>
__device__ __forceinline__ void block_weighted_cov(int N, const double* w, const double* m, Load load, double* out,
                                                   double* vlds, double* tmp)
{
    constexpr int NE = NV * (NV + 1) / 2;
    constexpr int NPASS = (NE + VSUM_MAX - 1) / VSUM_MAX;
    constexpr int CH = (NE + NPASS - 1) / NPASS;
    constexpr TriIndex<NV> tri{};
    const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
        const int c0 = pass * CH;
        int ea[CH], ec[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int t = c0 + e < NE ? c0 + e : NE - 1;
            ea[e] = tri.row[t];
            ec[e] = tri.col[t];
        }
        double acc[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) acc[e] = 0.0;
        for (int i = tid; i < N; i += nthr) {
            double z[NV];
            load(i, z);
#pragma unroll
            for (int v = 0; v < NV; ++v) z[v] -= m[v];
            const double wi = w[i];
#pragma unroll
            for (int e = 0; e < CH; ++e) acc[e] += wi * z[ea[e]] * z[ec[e]];
        }
        block_sum_vec<CH>(acc, vlds, tmp);
        if (tid < CH && c0 + tid < NE) {
            out[ea[tid] * NV + ec[tid]] = tmp[tid];
            out[ec[tid] * NV + ea[tid]] = tmp[tid];
        }
        __syncthreads();
    }
}

template <int D>
__global__ void __launch_bounds__(OUTER_BLOCK) k_outer(OuterArrays o, OuterParams p, const uint64_t* seeds)
{
    constexpr int D2 = 2 * D;
    const int r = (int)blockIdx.x;
    const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
    const int N = p.N;
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
    __shared__ double vlds[OUTER_WAVES * VSUM_MAX];
    __shared__ double mu[D2], cov[D2 * D2], A[D * D], LS[D * D], Lq[D * D], cth[D * D];
    __shared__ double est[VSUM_MAX];
    __shared__ int fit_ok;
    for (int e = tid; e < D * D; e += nthr) Lq[e] = p.lrw[e];
    if (tid == 0 && o.psteps_at) o.psteps_at[(size_t)r * p.K + (k - 1)] = o.psteps[r];
    __syncthreads();

    // proposal of this iteration: the learned one or one with the population's covariance
    // (then its density is in o.logq)
    const bool learned = p.mlp && k >= 2 && uniform_bool(o.mlp_use[r] != 0);
    const bool drift = p.popcov && k >= 2;

    // ---------------- approximately optimal L-kernel (k > 1)
    // Without a usable fit (forward-kernel setting, or the fit rejected) the backward
    // kernel is the random walk's Gaussian read backwards, N(phi_{k-1}; phi_k, Sigma_RW):
    // normalised in phi_{k-1} for any proposal, the forward kernel of the random walk
    // (whose log q it cancels exactly), and it keeps a learned proposal's density in
    // the weight.
    bool use_fit = false;
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
        // weighted mean of z_i = (phi_i, phi_new_i)
        {
            double acc[D2];
#pragma unroll
            for (int e = 0; e < D2; ++e) acc[e] = 0.0;
            for (int i = tid; i < N; i += nthr) {
                const double om = exp(logw[i] - W0);
                wsc[i] = om;
#pragma unroll
                for (int e = 0; e < D; ++e) {
                    acc[e] += om * phi[(size_t)i * D + e];
                    acc[D + e] += om * phin[(size_t)i * D + e];
                }
            }
            block_sum_vec<D2>(acc, vlds, mu);
        }
        // weighted covariance of the joint (phi_{k-1}, phi_k)
        block_weighted_cov<D2>(
            N, wsc, mu,
            [&](int i, double* z) {
#pragma unroll
                for (int e = 0; e < D; ++e) {
                    z[e] = phi[(size_t)i * D + e];
                    z[D + e] = phin[(size_t)i * D + e];
                }
            },
            cov, vlds, est);
        for (int e = tid; e < D2 + D2 * D2; e += nthr)
            o.lkfit[(size_t)r * (D2 + D2 * D2) + e] = e < D2 ? mu[e] : cov[e - D2];
        if (tid == 0) {
            // numerical-rank floor: every Cholesky pivot must exceed LK_REL_FLOOR times
            // its coordinate's raw second moment, else the population is degenerate
            // to rounding and the fit is rejected
            double L22[D * D], S[D * D], fl[D2];
            for (int a2 = 0; a2 < D2; ++a2) fl[a2] = LK_REL_FLOOR * (cov[a2 * D2 + a2] + mu[a2] * mu[a2]);
            int ok = chol_lower(D, cov + D * D2 + D, D2, L22) == 0;
            for (int a2 = 0; ok && a2 < D; ++a2) ok = L22[a2 * D + a2] * L22[a2 * D + a2] > fl[D + a2];
            if (ok) {
                for (int rr = 0; rr < D; ++rr) {
                    double b[D];
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
                for (int a2 = 0; ok && a2 < D; ++a2) ok = LS[a2 * D + a2] * LS[a2 * D + a2] > fl[a2];
            }
            fit_ok = ok;
        }
        __syncthreads();
        use_fit = uniform_bool(fit_ok != 0);
        fallback = use_fit ? 0 : 1;
    }

    // ---------------- weight update (Eq. l_weights)
    uint64_t dead = 0;
    double mloc = -INFINITY;
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
                double xo[D], xn[D];
#pragma unroll
                for (int a2 = 0; a2 < D; ++a2) {
                    xo[a2] = phi[(size_t)i * D + a2];
                    xn[a2] = phin[(size_t)i * D + a2];
                }
                double lL;
                if (use_fit) {
                    double m[D];
#pragma unroll
                    for (int a2 = 0; a2 < D; ++a2) {
                        double s = mu[a2];
#pragma unroll
                        for (int c = 0; c < D; ++c) s += A[a2 * D + c] * (xn[c] - mu[D + c]);
                        m[a2] = s;
                    }
                    lL = mvn_logpdf<D>(xo, m, LS);
                } else {
                    lL = mvn_logpdf<D>(xo, xn, Lq);
                }
                const double lq = (learned || drift) ? o.logq[base + i] : mvn_logpdf<D>(xn, xo, Lq);
                v = v + (lL - lq);
            }
        }
        lwp[i] = v;
        dead += (v == -INFINITY);
        mloc = v > mloc ? v : mloc;
    }
    const double M = uniform_f64(block_max<double>(mloc, &red));
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

    // ---------------- normalisation (Eq. normalise_smc2), quantised weights, ESS
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
    // ESS (Eq. ess_smc2) and the estimates at iteration k (Eq. realised_estimates)
    {
        double acc[2 * D + 1];
#pragma unroll
        for (int e = 0; e < 2 * D + 1; ++e) acc[e] = 0.0;
        for (int i = tid; i < N; i += nthr) {
            const double wn = exp(lwp[i] - W);
            wsc[i] = wn;
            acc[2 * D] += wn * wn;
#pragma unroll
            for (int e = 0; e < D; ++e) {
                acc[e] += wn * thn[(size_t)i * D + e];
                acc[D + e] += wn * phin[(size_t)i * D + e];
            }
        }
        block_sum_vec<2 * D + 1>(acc, vlds, est);
    }
    const double s2 = est[2 * D];
    double mth[D], mph[D];
#pragma unroll
    for (int e = 0; e < D; ++e) {
        mth[e] = est[e];
        mph[e] = est[D + e];
    }
    __syncthreads();
    block_weighted_cov<D>(
        N, wsc, mth,
        [&](int i, double* z) {
#pragma unroll
            for (int e = 0; e < D; ++e) z[e] = thn[(size_t)i * D + e];
        },
        cth, vlds, est);
    const bool rs = uniform_bool(ess_below_half(q1, q2, N));
    if (tid == 0) {
        rec[0] = (double)k;
        rec[1] = 1.0 / s2;
        rec[2] = rs ? 1.0 : 0.0;
        rec[3] = (double)dead;
        rec[4] = (double)fallback;
        rec[5] = W;
        rec[p.rec_len - 2] = learned ? 1.0 : (drift ? (p.langevin ? 2.0 : 3.0) : 0.0);
        for (int a2 = 0; a2 < D; ++a2) {
            rec[6 + a2] = mth[a2];
            rec[6 + D + D * D + a2] = mph[a2];
        }
        for (int e = 0; e < D * D; ++e) rec[6 + D + e] = cth[e];
        o.status[r] = 0;
    }

    // ---------------- resampling (Sec. IV-B) and redistribution (Alg. 1)
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
#pragma unroll
        for (int d = 0; d < D; ++d) phi[(size_t)m * D + d] = phin[(size_t)s * D + d];
        lp[m] = lpn[s];
        ll[m] = lln[s];
        logw[m] = rs ? 0.0 : lwp[m];
        if (p.langevin)  // the score estimates travel with their samples
#pragma unroll
            for (int d = 0; d < D; ++d) o.score[((size_t)base + m) * D + d] = o.score_new[((size_t)base + s) * D + d];
    }
}

// The proposal covariance of the Langevin and population random-walk proposals at iteration
// k > 1: the weighted covariance of the proposing population (normalised weights
// exp(log w - W), W = log sum exp log w) and its
// lower Cholesky factor, the diagonal of the standard deviations (floored at 1e-6) when a
// pivot is not above 1e-12 of its coordinate's raw second moment. One workgroup per run;
// the normalised weights go to o.scratch (free between outer updates).
template <int D>
__global__ void __launch_bounds__(OUTER_BLOCK) k_pop_frame(OuterArrays o, OuterParams p)
{
    if (*o.k_dev < 2) return;
    const int r = (int)blockIdx.x;
    const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
    const int N = p.N;
    const size_t base = (size_t)r * N;
    const double* phi = o.phi + base * D;
    const double* logw = o.logw + base;
    double* wn = o.scratch + base;
    __shared__ RedLds red;
    __shared__ double vlds[OUTER_WAVES * VSUM_MAX];
    __shared__ double tmp[VSUM_MAX];
    __shared__ double c[D], C[D * D];
    double mx = -INFINITY;
    for (int i = tid; i < N; i += nthr) mx = logw[i] > mx ? logw[i] : mx;
    const double M = uniform_f64(block_max<double>(mx, &red));
    double sw[1] = {0.0};
    for (int i = tid; i < N; i += nthr) sw[0] += exp(logw[i] - M);
    block_sum_vec<1>(sw, vlds, tmp);
    const double W = M + log(tmp[0]);
    double acc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] = 0.0;
    for (int i = tid; i < N; i += nthr) {
        const double w = exp(logw[i] - W);
        wn[i] = w;
#pragma unroll
        for (int d = 0; d < D; ++d) acc[d] += w * phi[(size_t)i * D + d];
    }
    block_sum_vec<D>(acc, vlds, tmp);
    if (tid < D) c[tid] = tmp[tid];
    __syncthreads();
    block_weighted_cov<D>(
        N, wn, c,
        [&](int i, double* z) {
#pragma unroll
            for (int d = 0; d < D; ++d) z[d] = phi[(size_t)i * D + d];
        },
        C, vlds, tmp);
    if (tid == 0) {
        double F[D * D];
#pragma unroll
        for (int e = 0; e < D * D; ++e) F[e] = 0.0;
        bool ok = true;
        for (int j = 0; j < D && ok; ++j) {
            double sj = C[j * D + j];
            for (int q = 0; q < j; ++q) sj -= F[j * D + q] * F[j * D + q];
            ok = sj > 1e-12 * (C[j * D + j] + c[j] * c[j]);
            if (!ok) break;
            F[j * D + j] = sqrt(sj);
            for (int i2 = j + 1; i2 < D; ++i2) {
                double v = C[i2 * D + j];
                for (int q = 0; q < j; ++q) v -= F[i2 * D + q] * F[j * D + q];
                F[i2 * D + j] = v / F[j * D + j];
            }
        }
        if (!ok) {
#pragma unroll
            for (int e = 0; e < D * D; ++e) F[e] = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double sd = sqrt(C[a * D + a]);
                F[a * D + a] = sd > 1e-6 ? sd : 1e-6;
            }
        }
        double* out = o.pop_chol + (size_t)r * D * D;
#pragma unroll
        for (int e = 0; e < D * D; ++e) out[e] = F[e];
    }
}

hipError_t launch_begin_iteration(const OuterArrays& o, int32_t* queues, int n_queues, hipStream_t s)
{
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, s, o.k_dev, queues, n_queues);
    return hipGetLastError();
}

template <int D> static hipError_t launch_d(const OuterArrays& o, const OuterParams& p, const uint64_t* d_seeds,
                                            hipStream_t s, bool outer)
{
    if (outer) {
        hipLaunchKernelGGL(k_outer<D>, dim3((unsigned)p.R), dim3(OUTER_BLOCK), 0, s, o, p, d_seeds);
    } else {
        const int total = p.R * p.N;
        hipLaunchKernelGGL(k_propose<D>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, o, p, d_seeds);
    }
    return hipGetLastError();
}

static hipError_t dispatch(const OuterArrays& o, const OuterParams& p, const uint64_t* d_seeds, hipStream_t s,
                           bool outer)
{
    switch (p.D) {
    case 1: return launch_d<1>(o, p, d_seeds, s, outer);
    case 2: return launch_d<2>(o, p, d_seeds, s, outer);
    case 3: return launch_d<3>(o, p, d_seeds, s, outer);
    case 4: return launch_d<4>(o, p, d_seeds, s, outer);
    case 5: return launch_d<5>(o, p, d_seeds, s, outer);
    case 6: return launch_d<6>(o, p, d_seeds, s, outer);
    case 7: return launch_d<7>(o, p, d_seeds, s, outer);
    case 8: return launch_d<8>(o, p, d_seeds, s, outer);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_propose(const OuterArrays& o, const OuterParams& p, const uint64_t* d_seeds, hipStream_t s)
{
    return dispatch(o, p, d_seeds, s, false);
}

hipError_t launch_outer_update(const OuterArrays& o, const OuterParams& p, const uint64_t* d_seeds,
                               hipStream_t s)
{
    return dispatch(o, p, d_seeds, s, true);
}

template <int D> static hipError_t launch_frame_d(const OuterArrays& o, const OuterParams& p, hipStream_t s)
{
    hipLaunchKernelGGL(k_pop_frame<D>, dim3((unsigned)p.R), dim3(OUTER_BLOCK), 0, s, o, p);
    return hipGetLastError();
}

hipError_t launch_pop_frame(const OuterArrays& o, const OuterParams& p, hipStream_t s)
{
    switch (p.D) {
    case 1: return launch_frame_d<1>(o, p, s);
    case 2: return launch_frame_d<2>(o, p, s);
    case 3: return launch_frame_d<3>(o, p, s);
    case 4: return launch_frame_d<4>(o, p, s);
    case 5: return launch_frame_d<5>(o, p, s);
    case 6: return launch_frame_d<6>(o, p, s);
    case 7: return launch_frame_d<7>(o, p, s);
    case 8: return launch_frame_d<8>(o, p, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace smc2
