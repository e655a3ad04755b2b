// device_common.h — device building blocks of the particle filter (gfx950).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the
// run seed; every draw is a pure function of its logical coordinates, so results
// do not depend on the launch shape. Counter layout:
//   flows       (particle j, filter i, k<<16 | t, 1<<24 | draw b<<16 | call a)
//   PF resample (0, filter i, k<<16 | t, 2<<24)
//   prior       (sample i, 0, 1<<16, 3<<24 | coordinate d)
//   RW normal   (sample i, 0, k<<16, 4<<24 | coordinate d)
//   outer resample (0, 0, k<<16, 5<<24)
//   learned proposal: initial parameter p (p, 0, 0, 6<<24); training permutation
//   (k, epoch, which, 7<<24)
// Uniforms: u24(x) = (2(x>>9)+1) 2^-24 (exact in FP32); u53 = (2(x64>>12)+1) 2^-53.
//
// Precision: the particle filter works in `real` (float or double). Every
// transcendental is evaluated in FP64 and rounded to `real`, every other
// operation is one IEEE operation in `real` (the library is built with
// -ffp-contract=off), so a reimplementation that follows the same definitions
// reproduces each integer decision.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc2 {

enum : uint32_t { S_PF_PROP = 1u, S_PF_RS = 2u, S_PRIOR = 3u, S_RW = 4u, S_OUTER_RS = 5u, S_MLP_INIT = 6u,
                  S_MLP_PERM = 7u };

struct W4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ W4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return W4{c0, c1, c2, c3};
}

__device__ __forceinline__ float u24(uint32_t x) { return (float)(2u * (x >> 9) + 1u) * 0x1p-24f; }

__host__ __device__ __forceinline__ double u53(uint32_t lo, uint32_t hi)
{
    const uint64_t x = ((uint64_t)hi << 32) | lo;
    return (double)(2ull * (x >> 12) + 1ull) * 0x1p-53;
}

// Box-Muller on one Philox call, first output.
__device__ __forceinline__ double normal_call(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint64_t seed)
{
    const W4 w = philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double r = sqrt(-2.0 * log(u53(w.x, w.y)));
    return r * cos(6.283185307179586 * u53(w.z, w.w));
}

// ----------------------------------------------------------- precision helpers
template <typename real> __device__ __forceinline__ real rdiv(real a, real b);
template <> __device__ __forceinline__ float rdiv<float>(float a, float b) { return __fdiv_rn(a, b); }
template <> __device__ __forceinline__ double rdiv<double>(double a, double b) { return a / b; }
template <typename real> __device__ __forceinline__ real rsqrt_rn(real a);
// Correctly rounded FP32 square root: the FP64 square root of a float, rounded to
// float, is the correctly rounded result (53 > 2*24 + 2 bits); the FP32 hardware
// square root is only accurate to 1 ulp.
template <> __device__ __forceinline__ float rsqrt_rn<float>(float a) { return (float)__dsqrt_rn((double)a); }
template <> __device__ __forceinline__ double rsqrt_rn<double>(double a) { return __dsqrt_rn(a); }

// Stream of one binomial draw: flows counter without the call index.
struct DrawStream {
    uint32_t j, i, kt, b;
    uint32_t k0, k1;
    __device__ __forceinline__ W4 call(uint32_t a) const
    {
        return philox10(j, i, kt, (S_PF_PROP << 24) | (b << 16) | a, k0, k1);
    }
};

// ----------------------------------------------------------- binomial sampler
// 1/m for m = 1..128, correctly rounded in each precision (compile-time division).
template <typename real> struct RcpTable {
    real v[128];
    constexpr RcpTable() : v()
    {
        for (int i = 0; i < 128; ++i) v[i] = (real)1 / (real)(i + 1);
    }
};
static __constant__ RcpTable<float> c_rcp_f32;
static __constant__ RcpTable<double> c_rcp_f64;
template <typename real> __device__ __forceinline__ real rcp_int(int m);
template <> __device__ __forceinline__ float rcp_int<float>(int m) { return c_rcp_f32.v[m - 1]; }
template <> __device__ __forceinline__ double rcp_int<double>(int m) { return c_rcp_f64.v[m - 1]; }

// Sequential-search inversion of the Binomial(n, p) CDF for p <= 1/2, n p < 10:
// f_0 = (1-p)^n, f_{k+1} = f_k ((n-k) r) / (k+1), r = p/(1-p); stops at the first k
// whose running sum reaches u, when adding a term no longer changes the sum, or
// at k = min(n, 127).
// l1p = log1p(-p) in FP64 (hoisted by callers whose p is fixed per filter).
template <typename real>
__device__ __forceinline__ int32_t binom_inversion(int32_t n, real p, double l1p, uint32_t word)
{
    const real u = (real)u24(word);
    const real q = (real)1 - p;
    const real r = rdiv<real>(p, q);
    real f = (real)exp((double)n * l1p);
    real F = f;
    int32_t k = 0;
    const int32_t kcap = n < 127 ? n : 127;
    while (u > F && k < kcap) {
        real t = (real)(n - k) * r;
        t = t * rcp_int<real>(k + 1);
        f = f * t;
        k = k + 1;
        const real Fn = F + f;
        if (Fn == F) break;
        F = Fn;
    }
    return k;
}

// log(x!) for integer-valued x >= 0 in FP64: exact table below 16, Stirling's series
// for log Gamma(x+1) with terms up to (x+1)^-7 above (truncation error < 1e-14).
static __constant__ double c_lfact_tab[16] = {
    0.0, 0.0, 0.69314718055994530942, 1.7917594692280550008, 3.1780538303479456196, 4.7874917427820459942,
    6.5792512120101009951, 8.5251613610654143002, 10.604602902745250228, 12.801827480081469611,
    15.104412573075515295, 17.502307845873885839, 19.98721449566188615, 22.552163853123422886,
    25.1912211827386815, 27.899271383840891566};

__device__ __forceinline__ double lfact(double x)
{
    if (x < 16.0) return c_lfact_tab[(int)x];
    const double z = x + 1.0;
    const double r = 1.0 / z, r2 = r * r;
    const double series = r * (1.0 / 12.0 - r2 * (1.0 / 360.0 - r2 * (1.0 / 1260.0 - r2 * (1.0 / 1680.0))));
    return ((x + 0.5) * log(z) - z) + 0.91893853320467274178 + series;
}

// BTRS transformed rejection (W. Hoermann, J. Stat. Comput. Simul. 46, 1993) for
// p <= 1/2, n p >= 10. Constants, proposal index and squeeze in `real`; the centre
// n p + 1/2 split in FP64 into integer and fraction; the final acceptance test in
// FP64 on log-factorials. Attempt e uses words 2(e&1), 2(e&1)+1 of call e>>1.
// The three pieces below are shared by the per-draw sampler (binom_btrs) and the
// particle filter's pooled schedule, which defers final tests; both take identical
// decisions because each piece is a pure function of (n, p, k, words).
template <typename real> struct BtrsConst {
    real spq, bb, aa, vr, cf;
    int64_t ci;
};

template <typename real> __device__ __forceinline__ BtrsConst<real> btrs_setup(int32_t n, real p)
{
    BtrsConst<real> c;
    const real nr = (real)n;
    const real q = (real)1 - p;
    c.spq = rsqrt_rn<real>((nr * p) * q);
    c.bb = (real)1.15 + (real)2.53 * c.spq;
    c.aa = ((real)-0.0873 + (real)0.0248 * c.bb) + (real)0.01 * p;
    c.vr = (real)0.92 - rdiv<real>((real)4.2, c.bb);
    const double cc = (double)n * (double)p + 0.5;
    const double cfl = floor(cc);
    c.ci = (int64_t)cfl;
    c.cf = (real)(cc - cfl);
    return c;
}

enum : int { BTRS_OUT = 0, BTRS_ACCEPT = 1, BTRS_FINAL = 2 };

// One attempt from the uniform words (wu, wv): the candidate k, and whether it lies
// outside [0, n], is accepted by the squeeze, or needs the final test.
template <typename real>
__device__ __forceinline__ int btrs_try(const BtrsConst<real>& c, int32_t n, uint32_t wu, uint32_t wv, int64_t& k)
{
    const real u = (real)u24(wu) - (real)0.5;
    const real v = (real)u24(wv);
    const real us = (real)0.5 - (real)fabs((double)u);
    real t = (real)2 * c.aa;
    t = rdiv<real>(t, us);
    t = t + c.bb;
    t = t * u;
    t = t + c.cf;
    k = c.ci + (int64_t)floor((double)t);
    if (k < 0 || k > n) return BTRS_OUT;
    if (us >= (real)0.07 && v <= c.vr) return BTRS_ACCEPT;
    return BTRS_FINAL;
}

// The final acceptance test of candidate k (FP64).
template <typename real>
__device__ __forceinline__ bool btrs_final(const BtrsConst<real>& c, int32_t n, real p, int64_t k, uint32_t wu,
                                           uint32_t wv)
{
    const real u = (real)u24(wu) - (real)0.5;
    const real v = (real)u24(wv);
    const real us = (real)0.5 - (real)fabs((double)u);
    const real q = (real)1 - p;
    const double alpha = (2.83 + 5.1 / (double)c.bb) * (double)c.spq;
    const double lpq = log((double)p / (double)q);
    const double m = floor((double)(n + 1) * (double)p);
    const double h = lfact(m) + lfact((double)n - m);
    const double lhs = log((double)v * alpha / ((double)c.aa / ((double)us * (double)us) + (double)c.bb));
    const double rhs = ((h - lfact((double)k)) - lfact((double)(n - k))) + ((double)k - m) * lpq;
    return lhs <= rhs;
}

// the value returned when 256 attempts were all rejected: the mode
template <typename real> __device__ __forceinline__ int32_t btrs_mode(int32_t n, real p)
{
    return (int32_t)floor((double)(n + 1) * (double)p);
}

template <typename real>
__device__ __forceinline__ int32_t binom_btrs(int32_t n, real p, const DrawStream& s)
{
    const BtrsConst<real> c = btrs_setup<real>(n, p);
    W4 w{0u, 0u, 0u, 0u};
    for (int e = 0; e < 256; ++e) {
        if ((e & 1) == 0) w = s.call((uint32_t)(e >> 1));
        const uint32_t wu = (e & 1) ? w.z : w.x;
        const uint32_t wv = (e & 1) ? w.w : w.y;
        int64_t k = 0;
        const int r = btrs_try<real>(c, n, wu, wv, k);
        // The acceptance is merged as a flag and k is returned after the branch: the
        // form "if (quick || final(...)) return k" was miscompiled for gfx950 (the
        // register holding k was reused inside the final test on the accepting path).
        bool acc = r == BTRS_ACCEPT;
        if (r == BTRS_FINAL) acc = btrs_final<real>(c, n, p, k, wu, wv);
        if (acc) return (int32_t)k;
    }
    return btrs_mode<real>(n, p);
}

// Binomial(n, p). l1p, when not NaN, is log1p(-min(p, 1-p)) precomputed in FP64.
template <typename real>
__device__ __forceinline__ int32_t binomial(int32_t n, real p, const DrawStream& s, double l1p = NAN)
{
    if (n <= 0 || !(p > (real)0)) return 0;
    if (p >= (real)1) return n;
    const bool flip = p > (real)0.5;
    const real pp = flip ? (real)1 - p : p;
    int32_t k;
    if ((real)n * pp < (real)10) {
        const double lq = (l1p == l1p) ? l1p : log1p(-(double)pp);
        k = binom_inversion<real>(n, pp, lq, s.call(0u).x);
    } else {
        k = binom_btrs<real>(n, pp, s);
    }
    return flip ? n - k : k;
}

// Probability 1 - exp(-x) of leaving a compartment within a day at hazard x.
template <typename real> __device__ __forceinline__ real leave_prob(real x)
{
    return (real)(-expm1(-(double)x));
}

// ----------------------------------------------------------- observations (FP64)
enum : int { OBS_POIS_PREV = 0, OBS_POIS_INC = 1, OBS_NB_INC = 2 };

// The observation log-pmf split into a per-day constant (no particle dependence)
// and a per-particle part, both FP64:
//   Poisson  log g = [y log(lambda) - lambda] + [-lgamma(y+1)]
//   NB       log g = -[y log1p(r/mu) + r log1p(mu/r)] + [lgamma(y+r) - lgamma(r) - lgamma(y+1)]
// The constant scales every weight equally: it leaves the normalised weights
// unchanged and enters the likelihood increment once per day. The per-particle
// parts have no cancellation, so their rounding to the filter precision is well
// defined. A zero mean gives 0 for y = 0 and -inf otherwise.
__device__ __forceinline__ double obs_const(int obs, int32_t y, double r)
{
    if (obs == OBS_NB_INC) return (lgamma((double)y + r) - lgamma(r)) - lgamma((double)y + 1.0);
    return -lgamma((double)y + 1.0);
}

template <int OBS> __device__ __forceinline__ double obs_part(int32_t y, int32_t cnt, double r)
{
    if (cnt <= 0) return (y == 0) ? 0.0 : -INFINITY;
    const double mu = (double)cnt;
    if (OBS == OBS_NB_INC) return -((double)y * log1p(r / mu) + r * log1p(mu / r));
    return (double)y * log(mu) - mu;
}

// ----------------------------------------------------------- wave / block primitives
// Values that every thread of a workgroup computes identically (block reductions,
// items read from LDS) live in vector registers, so the compiler cannot tell that a
// branch on them is uniform; around workgroup barriers it may then restructure the
// control flow per lane (a persistent work loop was split so that threads other than
// the one that fetches the next item looped without it). Reading such a value through
// readfirstlane makes it a scalar, and branches on it uniform.
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ bool uniform_bool(bool v) { return __builtin_amdgcn_readfirstlane((int)v) != 0; }
__device__ __forceinline__ float uniform_f32(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform_f64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
// true in every lane of the workgroup's first wave, as a scalar (uniform) condition
__device__ __forceinline__ bool first_wave() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x) == 0; }
template <typename real> __device__ __forceinline__ real uniform_real(real v);
template <> __device__ __forceinline__ float uniform_real<float>(float v) { return uniform_f32(v); }
template <> __device__ __forceinline__ double uniform_real<double>(double v) { return uniform_f64(v); }

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }

template <typename T> __device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const T u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// inclusive scan within a wave
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v)
{
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t u = __shfl_up(v, o, 64);
        if (l >= o) v += u;
    }
    return v;
}

}  // namespace smc2
