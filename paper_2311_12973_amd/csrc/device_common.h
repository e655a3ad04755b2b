// device_common.h — device building blocks of the particle filter (gfx950).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the
// run seed; every draw is a pure function of its logical coordinates, so results
// do not depend on the launch shape. Counter layout:
//   flows       (particle j, filter i, k<<16 | t, 1<<24 | draw b<<16 | call a)
//   PF resample (0, filter i, k<<16 | t, 2<<24); multinomial: slots 2p, 2p+1 from
//                (p, filter i, k<<16 | t, 2<<24 | 1<<16)
//   prior       (sample i, 0, 1<<16, 3<<24 | coordinate d)
//   RW normal   (sample i, 0, k<<16, 4<<24 | coordinate d)
//   outer resample (0, 0, k<<16, 5<<24)
//   learned proposal: initial parameter p (p, 0, 0, 6<<24); training permutation
//   (k, epoch, which, 7<<24)
//   linear-Gaussian state noise (particle j, filter i, k<<16 | t, 8<<24); t = 0 draws
//   the initial state
// Uniforms: u24(x) = (2(x>>9)+1) 2^-24 (exact in FP32); u53 = (2(x64>>12)+1) 2^-53.
//
// Precision: the particle filter works in `real` (float or double). Every
// transcendental is defined as its FP64 value rounded to `real`, every other
// operation is one IEEE operation in `real` (the library is built with
// -ffp-contract=off), so a reimplementation that follows the same definitions
// reproduces each integer decision. Two pieces reach the same result in FP32: the
// square root (correctly rounded) and the BTRS final test's decision (FP32 with an
// error bound, FP64 near the boundary).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc2 {

enum : uint32_t { S_PF_PROP = 1u, S_PF_RS = 2u, S_PRIOR = 3u, S_RW = 4u, S_OUTER_RS = 5u, S_MLP_INIT = 6u,
                  S_MLP_PERM = 7u, S_LG = 8u };

struct W4 {
    uint32_t x, y, z, w;
};

// a ^ b ^ c. With V3 on the device, one three-input bitwise vector instruction (truth
// table 0x96) instead of two XORs; it is a vector instruction even for uniform inputs, so
// it is meant for counters that differ per lane, where the XORs are vector work anyway.
template <bool V3> __host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (V3) return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#endif
    return a ^ b ^ c;
}

// V3: the round XORs as three-input vector instructions (per-lane counters)
template <bool V3 = false>
__host__ __device__ __forceinline__ W4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3<V3>((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3<V3>((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return W4{c0, c1, c2, c3};
}

// (2 (x >> 9) + 1) 2^-24. One funnel shift puts k = x >> 9 under the exponent of 1.0,
// giving 1 + k 2^-23; subtracting 1 - 2^-24 leaves (2k + 1) 2^-24 exactly (the operands
// lie within a factor of two of each other, so the difference is exact).
__device__ __forceinline__ float u24(uint32_t x)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, x, 9u)) - 0x1.fffffep-1f;
}

__host__ __device__ __forceinline__ double u53(uint32_t lo, uint32_t hi)
{
    const uint64_t x = ((uint64_t)hi << 32) | lo;
    return (double)(2ull * (x >> 12) + 1ull) * 0x1p-53;
}

// Box-Muller on one Philox call, first output.
__device__ __forceinline__ double normal_key(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1)
{
    const W4 w = philox10(c0, c1, c2, c3, k0, k1);
    const double r = sqrt(-2.0 * log(u53(w.x, w.y)));
    return r * cos(6.283185307179586 * u53(w.z, w.w));
}

__device__ __forceinline__ double normal_call(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint64_t seed)
{
    return normal_key(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ----------------------------------------------------------- precision helpers
template <typename real> __device__ __forceinline__ real rdiv(real a, real b);
template <> __device__ __forceinline__ float rdiv<float>(float a, float b) { return __fdiv_rn(a, b); }
template <> __device__ __forceinline__ double rdiv<double>(double a, double b) { return a / b; }
template <typename real> __device__ __forceinline__ real rsqrt_rn(real a);
// Correctly rounded FP32 square root (the FP64 root rounded to FP32, as the reference
// takes it). sqrtf is the correctly rounded sequence on gfx950 (checked against the FP64
// root on every mantissa of [1, 4), which covers both exponent parities of all normal
// inputs); __fsqrt_rn is the 1-ulp hardware root and differs on 15% of inputs.
template <> __device__ __forceinline__ float rsqrt_rn<float>(float a) { return sqrtf(a); }
template <> __device__ __forceinline__ double rsqrt_rn<double>(double a) { return __dsqrt_rn(a); }

// Stream of one binomial draw: flows counter without the call index.
struct DrawStream {
    uint32_t j, i, kt, b;
    uint32_t k0, k1;
    __device__ __forceinline__ W4 call(uint32_t a) const
    {
        return philox10<true>(j, i, kt, (S_PF_PROP << 24) | (b << 16) | a, k0, k1);
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
// n p + 1/2 split in FP64 into integer and fraction; the final acceptance test is
// defined in FP64 on log-factorials (btrs_final) and decided FP32-first with an error
// bound (btrs_final_fast, btrs_decide). Attempt e uses words 2(e&1), 2(e&1)+1 of call e>>1.
// The three pieces below are shared by the per-draw sampler (binom_btrs) and the
// particle filter's pooled schedule, which defers final tests; both take identical
// decisions because each piece is a pure function of (n, p, k, words).
template <typename real> struct BtrsConst {
    real spq, bb, aa, vr, cf;
    int32_t ci;
};

// The set-up given its two costly values, spq = sqrt(n p q) and vr = 0.92 - 4.2 / bb.
template <typename real>
__device__ __forceinline__ BtrsConst<real> btrs_setup_from(int32_t n, real p, real spq, real vr)
{
    BtrsConst<real> c;
    c.spq = spq;
    c.bb = (real)1.15 + (real)2.53 * c.spq;
    c.aa = ((real)-0.0873 + (real)0.0248 * c.bb) + (real)0.01 * p;
    c.vr = vr;
    const double cc = (double)n * (double)p + 0.5;
    const double cfl = floor(cc);
    c.ci = (int32_t)cfl;
    c.cf = (real)(cc - cfl);
    return c;
}

template <typename real> __device__ __forceinline__ BtrsConst<real> btrs_setup(int32_t n, real p)
{
    const real spq = rsqrt_rn<real>(((real)n * p) * ((real)1 - p));
    const real bb = (real)1.15 + (real)2.53 * spq;
    return btrs_setup_from<real>(n, p, spq, (real)0.92 - rdiv<real>((real)4.2, bb));
}

enum : int { BTRS_OUT = 0, BTRS_ACCEPT = 1, BTRS_FINAL = 2 };

// One attempt from the uniform words (wu, wv): the candidate k, and whether it lies
// outside [0, n], is accepted by the squeeze, or needs the final test.
// a / b correctly rounded, for positive normal operands whose quotient needs no range
// scaling: a >= 2^-100, b in [2^-100, 2^100], a / b below 2^100. Then the scale steps of
// the general division sequence leave the operands unchanged and its fix-up step passes
// the value through, so the core below (reciprocal, one Newton step, quotient, two
// residual corrections, all FMAs) gives the same bits as the general division.
__device__ __forceinline__ float fdiv_rn_inrange(float a, float b)
{
    const float y0 = __builtin_amdgcn_rcpf(b);
    const float e = fmaf(-b, y0, 1.0f);
    const float y1 = fmaf(e, y0, y0);
    const float q0 = a * y1;
    const float r0 = fmaf(-b, q0, a);
    const float q1 = fmaf(r0, y1, q0);
    const float r1 = fmaf(-b, q1, a);
    return fmaf(r1, y1, q1);
}
template <typename real> __device__ __forceinline__ real rdiv_btrs(real a, real b) { return rdiv<real>(a, b); }
template <> __device__ __forceinline__ float rdiv_btrs<float>(float a, float b) { return fdiv_rn_inrange(a, b); }

template <typename real>
__device__ __forceinline__ int btrs_try(const BtrsConst<real>& c, int32_t n, uint32_t wu, uint32_t wv, int32_t& k)
{
    const real u = (real)u24(wu) - (real)0.5;
    const real v = (real)u24(wv);
    const real us = (real)0.5 - (real)fabs((double)u);
    real t = (real)2 * c.aa;
    // in range: 2a with a = -0.0873 + 0.0248 b + 0.01 p in [0.12, 1100] (b = 1.15 + 2.53 sqrt(npq),
    // npq > 9, n < 2^30), over us in [2^-24, 1/2]
    t = rdiv_btrs<real>(t, us);
    t = t + c.bb;
    t = t * u;
    t = t + c.cf;
    // beyond 2^30 in magnitude the candidate lies outside [0, n] either way (n < 2^30):
    // clamped there, the sum stays within int32 and the range check decides the same
    k = c.ci + (int32_t)fmin(fmax(floor(t), (real)-0x1p30), (real)0x1p30);
    if (k < 0 || k > n) return BTRS_OUT;
    if (us >= (real)0.07 && v <= c.vr) return BTRS_ACCEPT;
    return BTRS_FINAL;
}

// The final acceptance test of candidate k (FP64).
template <typename real>
__device__ __forceinline__ bool btrs_final(const BtrsConst<real>& c, int32_t n, real p, int32_t k, uint32_t wu,
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

// The same test evaluated in FP32 with a bound on its distance from the FP64
// evaluation above; returns 1 (accept), -1 (reject), or 0 when the FP32 value is
// too close to the boundary to decide (then the FP64 test decides). Exact algebra
// on the test: with m = floor((n+1)p), d = k - m, A = k+1, B = n-k+1 and
// lfact(x) = (x+1/2) log(x+1) - (x+1) + log(2 pi)/2 + fc(x), the FP64 right-hand side is
//   (m+1/2) log((m+1)/A) + (n-m+1/2) log((n-m+1)/B) + d log(p B / (q A))
//     + fc(m) + fc(n-m) - fc(k) - fc(n-k),
// whose first two terms are each about +-d and cancel. With x1 = -d/A, x2 = d/B,
// log((m+1)/A) = log1p(x1) and log((n-m+1)/B) = log1p(x2); for |x| <= 1/8,
// log1p(x) = x + g(x) with g from its alternating series (terms to x^10, truncation
// below 2^-28 |g|), and when both are that small the two linear parts add up to the
// cancellation-free d [(d - 1/2)/B + (d + 1/2)/A]. Larger |x| take the logarithm of
// the ratio, which is then at least 0.11 in magnitude. In the third term
// p B - q A = ((n+1)p - m) + p - d - 1 + ((1-p) - q) A (q is 1 - p rounded to FP32,
// as in the FP64 test) is formed in FP64 without cancellation. Reciprocals and
// base-2 logarithms are the hardware instructions (relative error below 2^-22 on
// gfx950), so every piece carries a relative error of a few tens of FP32 units at
// most and 2^-17 times the sum of the magnitudes bounds the FP32 error;
// 2^-46 (n+1)(1 + log2(n+2)) bounds the FP64 evaluation's own error (terms of size n ln n, a
// few roundings each). A decision taken outside both bounds is the FP64 decision.
// Needs n < 2^23 (integers exact in FP32).
static __constant__ float c_fc_tab[16] = {
    0.081061466795327f, 0.041340695955409f, 0.027677925684998f, 0.020790672103766f,
    0.016644691189821f, 0.013876128823073f, 0.011896709945893f, 0.010411265261974f,
    0.009255462182709f, 0.008330563433359f, 0.007573675487949f, 0.006942840107207f,
    0.006408994188003f, 0.005951370112758f, 0.005554733551964f, 0.005207655919605f};

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_ln(float x) { return __builtin_amdgcn_logf(x) * 0.693147181f; }

// fc(x): the table below 16, else the Stirling series 1/(12z) - 1/(360z^3), z = x+1
// (the next term, 1/(1260 z^5) < 6e-10, and rounding stay below 1e-8)
__device__ __forceinline__ float btrs_fc(int32_t x)
{
    if (x < 16) return c_fc_tab[x];
    const float r = fast_rcp((float)(x + 1));
    return r * (0.0833333333f - (r * r) * 0.00277777778f);
}

// g(x) = log1p(x) - x for |x| <= 1/8, alternating series through x^10
__device__ __forceinline__ float log1p_minus_x(float x)
{
    float h = -0.1f;
    h = fmaf(h, x, 0.11111111f);
    h = fmaf(h, x, -0.125f);
    h = fmaf(h, x, 0.14285714f);
    h = fmaf(h, x, -0.16666667f);
    h = fmaf(h, x, 0.2f);
    h = fmaf(h, x, -0.25f);
    h = fmaf(h, x, 0.33333333f);
    h = fmaf(h, x, -0.5f);
    return (x * x) * h;
}

template <typename real>
__device__ __forceinline__ int btrs_final_fast(const BtrsConst<real>& c, int32_t n, real p, int32_t k, uint32_t wu,
                                               uint32_t wv)
{
    if constexpr (sizeof(real) != 4) {
        return 0;
    } else {
        if (n >= (1 << 23)) return 0;
        const float u = u24(wu) - 0.5f;
        const float v = u24(wv);
        const float us = 0.5f - fabsf(u);
        const float q = 1.0f - p;
        const double mp = (double)(n + 1) * (double)p;  // exact: 24-bit times 24-bit
        const double mfl = floor(mp);
        const int32_t m = (int32_t)mfl;
        const int32_t ki = k;
        const int32_t d = ki - m;
        const float df = (float)d;
        const float A = (float)(ki + 1), B = (float)(n - ki + 1);
        const float rA = fast_rcp(A), rB = fast_rcp(B);
        const float mh = (float)m + 0.5f, nmh = (float)(n - m) + 0.5f;
        // (m+1/2) log((m+1)/A) + (n-m+1/2) log((n-m+1)/B)
        const float x1 = -df * rA, x2 = df * rB;
        const bool s1 = fabsf(x1) <= 0.125f, s2 = fabsf(x2) <= 0.125f;
        const float lin = (s1 && s2) ? df * ((df - 0.5f) * rB + (df + 0.5f) * rA)
                                     : (s1 ? mh * x1 : 0.0f) + (s2 ? nmh * x2 : 0.0f);
        const float b1 = mh * (s1 ? log1p_minus_x(x1) : fast_ln((float)(m + 1) * rA));
        const float b2 = nmh * (s2 ? log1p_minus_x(x2) : fast_ln((float)(n - m + 1) * rB));
        // d log(p B / (q A)), q = fl(1 - p) as in the FP64 test:
        // p B - q A = (fr + p - d - 1) + ((1 - p) - q) A
        const double dq = (1.0 - (double)p) - (double)q;  // exact
        const float num = (float)((((mp - mfl) + (double)p) - (double)(d + 1)) + dq * (double)A);
        const float y3 = num * fast_rcp(q * A);
        const float l3 = fabsf(y3) <= 0.125f ? y3 + log1p_minus_x(y3)
                         : (y3 < -0.5f ? -fast_ln(1.0f - num * fast_rcp(p * B)) : fast_ln(1.0f + y3));
        const float t3 = df * l3;
        const float f = (btrs_fc(m) + btrs_fc(n - m)) - (btrs_fc(ki) + btrs_fc(n - ki));
        // left-hand side log(v alpha / (aa / us^2 + bb))
        const float alpha = (2.83f + 5.1f * fast_rcp(c.bb)) * c.spq;
        const float den = c.aa * fast_rcp(us * us) + c.bb;
        const float lhs = fast_ln((v * alpha) * fast_rcp(den));
        const float D = (((lin + b1) + b2) + t3 + f) - lhs;
        const float nf = (float)(n + 1);
        const float E = 0x1p-17f * (((((fabsf(lin) + fabsf(b1)) + fabsf(b2)) + fabsf(t3)) + fabsf(f)) + fabsf(lhs) + 1.0f) +
                        0x1p-46f * nf * (1.0f + __builtin_amdgcn_logf(nf + 1.0f));
        return D > E ? 1 : (D < -E ? -1 : 0);
    }
}

// btrs_final as a call, for the per-draw sampler: the FP64 test is taken only near the
// boundary of the FP32 one, and kept out of line its registers do not weigh on the
// draw loop around it.
template <typename real>
__device__ __attribute__((noinline)) bool btrs_final_call(const BtrsConst<real> c, int32_t n, real p, int32_t k,
                                                          uint32_t wu, uint32_t wv)
{
    return btrs_final<real>(c, n, p, k, wu, wv);
}

// The acceptance decision of a candidate that needs the final test: FP32 first, the
// FP64 test only when the FP32 value cannot decide.
template <typename real>
__device__ __forceinline__ bool btrs_decide(const BtrsConst<real>& c, int32_t n, real p, int32_t k, uint32_t wu,
                                            uint32_t wv)
{
    const int f = btrs_final_fast<real>(c, n, p, k, wu, wv);
    bool acc = f > 0;
    if (f == 0) acc = btrs_final_call<real>(c, n, p, k, wu, wv);
    return acc;
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
        int32_t k = 0;
        const int r = btrs_try<real>(c, n, wu, wv, k);
        // The acceptance is merged as a flag and k is returned after the branch: the
        // form "if (quick || final(...)) return k" was miscompiled for gfx950 (the
        // register holding k was reused inside the final test on the accepting path).
        bool acc = r == BTRS_ACCEPT;
        if (r == BTRS_FINAL) {
            const int f = btrs_final_fast<real>(c, n, p, k, wu, wv);
            acc = f > 0;
            if (f == 0) acc = btrs_final_call<real>(c, n, p, k, wu, wv);
        }
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
enum : int { OBS_POIS_PREV = 0, OBS_POIS_INC = 1, OBS_NB_INC = 2, OBS_GAUSS = 3 };

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
