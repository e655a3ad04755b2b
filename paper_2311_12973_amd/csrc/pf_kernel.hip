// pf_kernel.hip — the batch of particle filters (Sec. II) on gfx950.
//
// One workgroup runs one particle filter: it owns the filter's N_x particles for
// all T days. Thread t works on particles t, t + blockDim, ... whose compartment
// counts and log-weights stay in LDS, so the only HBM traffic is theta, the
// observations (L2-resident, shared by all filters) and one log-likelihood per
// filter. Per day:
//   1. propagate every particle through the chain-binomial model (Sec. V-A),
//      flows drawn from counter-based Philox streams (particle, filter, k, t, draw);
//   2. weight update a = lw + log g(y_t | x_t) - c_t (Sec. II, bootstrap proposal;
//      c_t, the particle-independent part of log g, is carried separately);
//   3. block max m, then w = exp(a - m) in FP64; the FP64 block sum S gives the
//      likelihood increment m + log S - log S_prev + c_t (the mean unnormalised
//      weight of Sec. II, accumulated in FP64);
//   4. if ESS < N_x/2 (exact integer test on the quantised weights) and t < T:
//      integer systematic resampling (LDS scan + search), gather of the counts
//      through LDS, log-weights reset (every particle gets the mean weight).
// The scalar linear-Gaussian model, whose likelihood the Kalman filter gives in
// closed form, runs through the same steps (FP64 only): its state is one FP64 value
// per particle, held in LDS as two 32-bit words, and its noise comes from Box-Muller
// on the counter (particle j, filter i, k<<16 | t, 8<<24).
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "block_ops.h"
#include "pf_kernel.h"

namespace smc2 {

template <int MODEL> struct ModelShape;
template <> struct ModelShape<MODEL_SIR> { static constexpr int NC = 2, NG = 1; };
template <> struct ModelShape<MODEL_SEIR> { static constexpr int NC = 3, NG = 1; };
template <> struct ModelShape<MODEL_AGE> { static constexpr int NC = 12, NG = 4; };
// linear-Gaussian: the FP64 state and the FP64 observation each take two 32-bit words
template <> struct ModelShape<MODEL_LG> { static constexpr int NC = 2, NG = 2; };

// Per-filter constants of the transition kernel, rounded once to `real`.
template <typename real> struct MConst {
    real cinf;      // beta / N_pop
    real p_ei;      // 1 - exp(-sigma)
    real p_ir;      // 1 - exp(-gamma)
    real cs[4][4];  // beta s_g C_gh / N_h  (age-structured)
    double l1p_ei;  // log1p(-min(p_ei, 1-p_ei)), log1p(-min(p_ir, 1-p_ir)) in FP64
    double l1p_ir;
    double r;       // negative-binomial dispersion
    int32_t x0[12]; // initial compartment counts
    double ar, sq, sr, m0, s0;  // linear-Gaussian: x_t = ar x_{t-1} + sq e_t, y_t = x_t + sr d_t,
                                // x_0 = m0 + s0 e_0
};

template <typename real> __device__ __forceinline__ double l1p_of(real p)
{
    const real pp = p > (real)0.5 ? (real)1 - p : p;
    return log1p(-(double)pp);
}

template <typename real, int MODEL>
__device__ __forceinline__ void model_setup(const PFArgs& a, const double* th, MConst<real>& mc)
{
    if constexpr (MODEL == MODEL_LG) {
        mc.ar = uniform_f64(th[0]);
        mc.sq = uniform_f64(th[1]);
        mc.sr = uniform_f64(th[2]);
        mc.m0 = a.fx[0];
        mc.s0 = a.fx[1];
        return;
    }
    if (MODEL == MODEL_SIR) {
        const int32_t i0 = (int32_t)a.fx[0];
        mc.cinf = (real)(th[0] / a.n_pop);
        mc.p_ir = (real)(-expm1(-th[1]));
        mc.p_ei = (real)0;
        mc.r = 0.0;
        mc.x0[0] = (int32_t)a.n_pop - i0;
        mc.x0[1] = i0;
    } else if (MODEL == MODEL_SEIR) {
        mc.r = (a.D >= 5) ? th[4] : a.fx[0];
        mc.cinf = (real)(th[0] / a.n_pop);
        mc.p_ei = (real)(-expm1(-th[1]));
        mc.p_ir = (real)(-expm1(-th[2]));
        double i0 = floor(th[3] * a.n_pop + 0.5);
        i0 = i0 < 1.0 ? 1.0 : (i0 > a.n_pop ? a.n_pop : i0);
        mc.x0[0] = (int32_t)(a.n_pop - i0);
        mc.x0[1] = 0;
        mc.x0[2] = (int32_t)i0;
    } else {
        mc.r = th[4];
        mc.cinf = (real)0;
        mc.p_ei = (real)(-expm1(-th[1]));
        mc.p_ir = (real)(-expm1(-th[2]));
        const double s[4] = {1.0, th[5], th[6], th[7]};
        double ng[4];
        for (int g = 0; g < 4; ++g) ng[g] = floor(a.fx[16 + g] * a.n_pop + 0.5);
        for (int g = 0; g < 4; ++g)
            for (int h = 0; h < 4; ++h) mc.cs[g][h] = (real)(((th[0] * s[g]) * a.fx[4 * g + h]) / ng[h]);
        for (int g = 0; g < 4; ++g) {
            double i0 = floor(th[3] * ng[g] + 0.5);
            i0 = i0 < 1.0 ? 1.0 : (i0 > ng[g] ? ng[g] : i0);
            mc.x0[3 * g] = (int32_t)(ng[g] - i0);
            mc.x0[3 * g + 1] = 0;
            mc.x0[3 * g + 2] = (int32_t)i0;
        }
    }
    mc.l1p_ei = l1p_of<real>(mc.p_ei);
    mc.l1p_ir = l1p_of<real>(mc.p_ir);
    if (MODEL == MODEL_AGE) {
        // every thread computed the same values: held in scalar registers, they leave
        // the vector registers to the draws
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int h = 0; h < 4; ++h) mc.cs[g][h] = uniform_real<real>(mc.cs[g][h]);
        mc.p_ei = uniform_real<real>(mc.p_ei);
        mc.p_ir = uniform_real<real>(mc.p_ir);
        mc.l1p_ei = uniform_f64(mc.l1p_ei);
        mc.l1p_ir = uniform_f64(mc.l1p_ir);
        mc.r = uniform_f64(mc.r);
    }
}

// ------------------------------------------------------------ score (Fisher's identity)
// Score coordinates kept per particle (on the natural parameters), as FP64 values in
// pairs of 32-bit LDS words after the counts: column d at sw[2d cap + j] (low word) and
// sw[(2d + 1) cap + j] (high word), so the resampling gather moves them with the counts.
template <int MODEL> struct ScoreDims { static constexpr int NS = 0; };
template <> struct ScoreDims<MODEL_SIR> { static constexpr int NS = 2; };   // beta, gamma
template <> struct ScoreDims<MODEL_SEIR> { static constexpr int NS = 5; };  // beta, sigma, gamma, iota (0), r
template <> struct ScoreDims<MODEL_LG> { static constexpr int NS = 3; };    // a, sigma_x, sigma_y

__device__ __forceinline__ double lds_f64(const int32_t* w, int cap, int j) { return __hiloint2double(w[cap + j], w[j]); }
__device__ __forceinline__ void lds_add_f64(int32_t* w, int cap, int j, double v)
{
    const double x = __hiloint2double(w[cap + j], w[j]) + v;
    w[j] = __double2loint(x);
    w[cap + j] = __double2hiint(x);
}

// d log Bin(k; n, p) / d h for p = 1 - exp(-h): (k - n p) / p, and -n at p = 0 (k = 0 then)
template <typename real> __device__ __forceinline__ double flow_score(int32_t n, real p, int32_t k)
{
    return p > (real)0 ? ((double)k - (double)n * (double)p) / (double)p : -(double)n;
}

// psi(x), x > 0, in FP64: the recurrence psi(x) = psi(x + 1) - 1/x up to x >= 10, then the
// asymptotic expansion ln x - 1/(2x) - sum_{k=1..7} B_2k / (2k x^2k) (Bernoulli numbers)
__device__ __noinline__ double digamma_f64(double x)
{
    double acc = 0.0;
    while (x < 10.0) {
        acc = acc - 1.0 / x;
        x = x + 1.0;
    }
    const double r = 1.0 / x, r2 = r * r;
    const double tail =
        r2 * (1.0 / 12 - r2 * (1.0 / 120 - r2 * (1.0 / 252 - r2 * (1.0 / 240 - r2 * (1.0 / 132 - r2 * (691.0 / 32760 - r2 * (1.0 / 12)))))));
    return acc + ((log(x) - 0.5 * r) - tail);
}

// what particle_day needs for the score: the score words, N_pop, the day's
// psi(y_t + r) - psi(r), and whether r is a parameter
struct ScoreDay {
    int32_t* sw;
    double n_pop;
    double dpsi;
    bool nr;
};

// Issue priority of a wave from its progress through the day's draws, step of total (a
// particle pass times the model's draw groups): 3 in the first quarter of its work, down
// to 0 in the last. The waves of a filter meet at a barrier after the draws, and their
// draws take different times (attempts, final tests, inversion lengths differ): a wave
// that has done less of its day outranks one near its end, so the laggards catch up and
// the barrier waits shrink (age-structured SEIR, N_x = 2048, T = 365, one filter per CU:
// 1.45 -> 1.36 s per launch of 16384 filters, VALU busy 0.91 -> 0.99). Results do not
// depend on it: it only orders instruction issue.
__device__ __forceinline__ void progress_priority(int step, int total)
{
    const int q = uniform_i32((4 * step) / total);
    if (q <= 0) __builtin_amdgcn_s_setprio(3);
    else if (q == 1) __builtin_amdgcn_s_setprio(2);
    else if (q == 2) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// Draw groups of a particle-day, the steps of progress_priority: SIR's two draws, SEIR's
// three, the age-structured model's four groups, the linear-Gaussian model's one normal.
template <int MODEL> struct DrawGroups {
    static constexpr int G = MODEL == MODEL_SIR ? 2 : (MODEL == MODEL_SEIR ? 3 : (MODEL == MODEL_AGE ? 4 : 1));
};

// One day of the chain-binomial model for particle j, whose counts live in LDS
// (st[c * cap + j]); flows drawn from the previous day's state. Draw index b:
// SIR (S->I, I->R) = (0, 1); SEIR (S->E, E->I, I->R) = (0, 1, 2); age-structured
// group g: 3g, 3g+1, 3g+2 (the draw index equals the index of the compartment the
// flow leaves). One copy of the sampler per model: the draws of a day run in a
// loop. Returns the per-particle part of log g(y_t | x_t) in FP64. With SCORE it adds
// the day's complete-data score to the particle's: per flow d log Bin / d h times
// d h / d theta (I / N_pop for beta, 1 for sigma and gamma), d log g / d r, and for the
// linear-Gaussian model the derivatives of its two Gaussian densities. With ptotal > 0
// each draw group first sets the wave's issue priority (progress_priority, step pbase +
// group of ptotal).
template <typename real, int MODEL, int OBS, bool SCORE = false>
__device__ __forceinline__ double particle_day(const MConst<real>& mc, int32_t* st, int cap, int j,
                                               DrawStream ds, const int32_t* yt, const ScoreDay& sd = ScoreDay{},
                                               int pbase = 0, int ptotal = 0)
{
    if constexpr (MODEL == MODEL_LG) {
        // x_t = ar x_{t-1} + sq e_t; log g = -z^2 / 2 with z = (y_t - x_t) / sr (the
        // constant -log sr - log(2 pi) / 2 goes with the day's constant)
        if (ptotal > 0) progress_priority(pbase, ptotal);
        const double x = __hiloint2double(st[cap + j], st[j]);
        const double e = normal_key(ds.j, ds.i, ds.kt, S_LG << 24, ds.k0, ds.k1);
        const double x1 = mc.ar * x + mc.sq * e;
        st[j] = __double2loint(x1);
        st[cap + j] = __double2hiint(x1);
        const double z = (__hiloint2double(yt[1], yt[0]) - x1) / mc.sr;
        if constexpr (SCORE) {
            lds_add_f64(sd.sw, cap, j, (e * x) / mc.sq);
            lds_add_f64(sd.sw + 2 * cap, cap, j, (e * e - 1.0) / mc.sq);
            lds_add_f64(sd.sw + 4 * cap, cap, j, (z * z - 1.0) / mc.sr);
        }
        return -0.5 * z * z;
    }
    if (MODEL == MODEL_SIR) {
        const int32_t S = st[j], I = st[cap + j];
        const real p_si = leave_prob<real>(mc.cinf * (real)I);
        int32_t nsi = 0, nir = 0;
#pragma nounroll
        for (int b = 0; b < 2; ++b) {
            if (ptotal > 0) progress_priority(pbase + b, ptotal);
            ds.b = (uint32_t)b;
            const int32_t v = binomial<real>(b == 0 ? S : I, b == 0 ? p_si : mc.p_ir, ds, b == 0 ? NAN : mc.l1p_ir);
            nsi = b == 0 ? v : nsi;
            nir = b == 1 ? v : nir;
        }
        const int32_t I1 = I + nsi - nir;
        st[j] = S - nsi;
        st[cap + j] = I1;
        if constexpr (SCORE) {
            lds_add_f64(sd.sw, cap, j, flow_score<real>(S, p_si, nsi) * ((double)I / sd.n_pop));
            lds_add_f64(sd.sw + 2 * cap, cap, j, flow_score<real>(I, mc.p_ir, nir));
        }
        return obs_part<OBS>(yt[0], OBS == OBS_POIS_PREV ? I1 : nsi, mc.r);
    } else if (MODEL == MODEL_SEIR) {
        const int32_t S = st[j], E = st[cap + j], I = st[2 * cap + j];
        const real p_se = leave_prob<real>(mc.cinf * (real)I);
        int32_t nse = 0, nei = 0, nir = 0;
#pragma nounroll
        for (int b = 0; b < 3; ++b) {
            if (ptotal > 0) progress_priority(pbase + b, ptotal);
            ds.b = (uint32_t)b;
            const int32_t n = b == 0 ? S : (b == 1 ? E : I);
            const real p = b == 0 ? p_se : (b == 1 ? mc.p_ei : mc.p_ir);
            const double l1p = b == 0 ? NAN : (b == 1 ? mc.l1p_ei : mc.l1p_ir);
            const int32_t v = binomial<real>(n, p, ds, l1p);
            nse = b == 0 ? v : nse;
            nei = b == 1 ? v : nei;
            nir = b == 2 ? v : nir;
        }
        const int32_t I1 = I + nei - nir;
        st[j] = S - nse;
        st[cap + j] = E + nse - nei;
        st[2 * cap + j] = I1;
        if constexpr (SCORE) {
            lds_add_f64(sd.sw, cap, j, flow_score<real>(S, p_se, nse) * ((double)I / sd.n_pop));
            lds_add_f64(sd.sw + 2 * cap, cap, j, flow_score<real>(E, mc.p_ei, nei));
            lds_add_f64(sd.sw + 4 * cap, cap, j, flow_score<real>(I, mc.p_ir, nir));
            // d/dr log NB(y; mu, r) = psi(y + r) - psi(r) - log1p(mu / r) + (mu - y) / (r + mu)
            if (sd.nr && nei > 0) {
                const double mu = (double)nei, r = mc.r;
                lds_add_f64(sd.sw + 8 * cap, cap, j, (sd.dpsi - log1p(mu / r)) + (mu - (double)yt[0]) / (r + mu));
            }
        }
        return obs_part<OBS>(yt[0], OBS == OBS_POIS_PREV ? I1 : nei, mc.r);
    } else {
        // forces of infection from the previous day's infected counts
        real pse0, pse1, pse2, pse3;
        {
            real acc[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                acc[g] = (real)0;
#pragma unroll
                for (int h = 0; h < 4; ++h) acc[g] = acc[g] + mc.cs[g][h] * (real)st[(3 * h + 2) * cap + j];
            }
            pse0 = leave_prob<real>(acc[0]);
            pse1 = leave_prob<real>(acc[1]);
            pse2 = leave_prob<real>(acc[2]);
            pse3 = leave_prob<real>(acc[3]);
        }
        double lg = 0.0;
#pragma nounroll
        for (int g = 0; g < 4; ++g) {
            if (ptotal > 0) progress_priority(pbase + g, ptotal);
            const int32_t S = st[(3 * g) * cap + j], E = st[(3 * g + 1) * cap + j], I = st[(3 * g + 2) * cap + j];
            const real p_se = g == 0 ? pse0 : (g == 1 ? pse1 : (g == 2 ? pse2 : pse3));
            int32_t nse = 0, nei = 0, nir = 0;
#pragma nounroll
            for (int b = 0; b < 3; ++b) {
                ds.b = (uint32_t)(3 * g + b);
                const int32_t n = b == 0 ? S : (b == 1 ? E : I);
                const real p = b == 0 ? p_se : (b == 1 ? mc.p_ei : mc.p_ir);
                const double l1p = b == 0 ? NAN : (b == 1 ? mc.l1p_ei : mc.l1p_ir);
                const int32_t v = binomial<real>(n, p, ds, l1p);
                nse = b == 0 ? v : nse;
                nei = b == 1 ? v : nei;
                nir = b == 2 ? v : nir;
            }
            const int32_t I1 = I + nei - nir;
            st[(3 * g) * cap + j] = S - nse;
            st[(3 * g + 1) * cap + j] = E + nse - nei;
            st[(3 * g + 2) * cap + j] = I1;
            lg = lg + obs_part<OBS>(yt[g], OBS == OBS_POIS_PREV ? I1 : nei, mc.r);
        }
        return lg;
    }
}

// ---------------------------------------------------------------- pooled schedule
// SIR and SEIR draw a day's flows as a pool of work items instead of one particle
// after another. The flows of a day depend only on the previous day's counts, so the
// draws of all the filter's particles are independent items (particle j, draw b),
// handed out from one workgroup-wide list through an LDS counter. Every round each
// free lane of a wave takes the next item (trivial draws finish at once, inversion
// draws within the round), and every lane with a BTRS item makes one attempt. An
// attempt outside [0, n] is retried next round; one that needs the final acceptance
// test goes to the wave's queue in LDS and the lane moves on. When 64 tests are
// queued the wave runs them with all lanes busy (FP32 first, FP64 only near the
// boundary), and a candidate that fails continues with its next attempts in its lane.
// The last tests of the day, fewer than 64, each take several lanes that evaluate the
// draw's following attempts at once. A wave would otherwise pay for the final test
// whenever any one of its lanes needs it, which is nearly every round. Every attempt
// is a function of its Philox coordinates alone, so the flows equal the per-draw
// schedule's whichever lane or wave draws them. Flows go to flows[b * cap + j] (the
// quantised-weight and gather buffers, free during propagation); the counts are
// updated once every wave has finished the day's draws.
constexpr int POOL_CAP = 128;  // < 64 entries remain after the flushes; one round adds at most 64

template <typename real> struct WavePool {
    uint32_t id[POOL_CAP];  // j | b << 12 | flip << 15 | attempt << 16
    int32_t n[POOL_CAP];
    int32_t k[POOL_CAP];
    uint32_t wu[POOL_CAP];
    uint32_t wv[POOL_CAP];
    real p[POOL_CAP];
    real spq[POOL_CAP];  // the draw's BTRS set-up values sqrt(n p q) and v_r, so that the
    real vr[POOL_CAP];   // test does not redo the root and the division
};

template <typename real> __device__ __forceinline__ void pool_store(WavePool<real>* q, int s, uint32_t id,
                                                                     int32_t n, int32_t k, uint32_t wu,
                                                                     uint32_t wv, real p, const BtrsConst<real>& c)
{
    q->id[s] = id;
    q->n[s] = n;
    q->k[s] = k;
    q->wu[s] = wu;
    q->wv[s] = wv;
    q->p[s] = p;
    q->spq[s] = c.spq;
    q->vr[s] = c.vr;
}

__device__ __forceinline__ uint64_t lanes_below() { return __lanemask_lt(); }

// Starts item (j, b): n and p from the day-start counts. Returns true with the flow
// in res when the draw finishes without BTRS (n = 0, p in {0, 1}, inversion).
template <typename real, int MODEL>
__device__ __forceinline__ bool item_begin(const MConst<real>& mc, const int32_t* st, int cap, int j, int b,
                                           const DrawStream& ds, int32_t& n, real& pp, bool& flip,
                                           BtrsConst<real>& c, int32_t& res)
{
    constexpr int ND = ModelShape<MODEL>::NC;
    n = st[b * cap + j];
    real p;
    double l1p;
    if (b == 0) {
        p = leave_prob<real>(mc.cinf * (real)st[(ND - 1) * cap + j]);
        l1p = NAN;
    } else if (b == ND - 1) {
        p = mc.p_ir;
        l1p = mc.l1p_ir;
    } else {
        p = mc.p_ei;
        l1p = mc.l1p_ei;
    }
    if (n <= 0 || !(p > (real)0)) {
        res = 0;
        return true;
    }
    if (p >= (real)1) {
        res = n;
        return true;
    }
    flip = p > (real)0.5;
    pp = flip ? (real)1 - p : p;
    if ((real)n * pp < (real)10) {
        const double lq = (l1p == l1p) ? l1p : log1p(-(double)pp);
        const int32_t k = binom_inversion<real>(n, pp, lq, ds.call(0u).x);
        res = flip ? n - k : k;
        return true;
    }
    c = btrs_setup<real>(n, pp);
    return false;
}

template <typename real, int MODEL>
__device__ void draws_pooled(const MConst<real>& mc, const int32_t* st, int32_t* flows, int cap, int nx,
                             WavePool<real>* q, uint32_t filt, uint32_t kt, uint32_t k0, uint32_t k1, int* wg_next)
{
    constexpr int ND = ModelShape<MODEL>::NC;
    const int lane = lane_id();
    const int F = ND * cap;           // items of the workgroup, b-major: item f is (b, j) = (f / cap, f % cap)
    const uint64_t below = lanes_below();
    int fq = 0;                       // wave-uniform: queued final tests
    bool exhausted = false;           // wave-uniform: the workgroup's item list is used up
    bool busy = false;
    int32_t j = 0, b = 0, n = 0, e = 0;
    bool flip = false;
    real pp = (real)0;
    BtrsConst<real> c{};
    for (;;) {
        // 1. free lanes take the next items of the workgroup's list (the waves share it,
        //    so a wave whose draws needed fewer attempts takes more items)
        const uint64_t freem = __ballot(!busy);
        const int nfree = __popcll(freem);
        int base = 0;
        if (!exhausted && nfree > 0) {
            if (lane == 0) base = atomicAdd(wg_next, nfree);
            base = uniform_i32(base);  // lane 0's value: every lane is active here
            if (base + nfree >= F) exhausted = true;
        } else {
            base = F;
        }
        if (!busy) {
            const int f = base + __popcll(freem & below);
            if (f < F) {
                b = (f >= cap ? 1 : 0) + (ND > 2 && f >= 2 * cap ? 1 : 0);
                j = f - b * cap;
                if (j < nx) {
                    int32_t res;
                    const DrawStream ds{(uint32_t)j, filt, kt, (uint32_t)b, k0, k1};
                    if (item_begin<real, MODEL>(mc, st, cap, j, b, ds, n, pp, flip, c, res)) {
                        flows[b * cap + j] = res;
                    } else {
                        busy = true;
                        e = 0;
                    }
                }
            }
        }
        // 2. one BTRS attempt per busy lane
        bool push = false;
        int32_t kk = 0;
        uint32_t wu = 0, wv = 0;
        if (busy) {
            if (e >= 256) {
                const int32_t r = btrs_mode<real>(n, pp);
                flows[b * cap + j] = flip ? n - r : r;
                busy = false;
            } else {
                const W4 w = DrawStream{(uint32_t)j, filt, kt, (uint32_t)b, k0, k1}.call((uint32_t)(e >> 1));
                wu = (e & 1) ? w.z : w.x;
                wv = (e & 1) ? w.w : w.y;
                const int r = btrs_try<real>(c, n, wu, wv, kk);
                if (r == BTRS_ACCEPT) {
                    flows[b * cap + j] = flip ? n - (int32_t)kk : (int32_t)kk;
                    busy = false;
                } else if (r == BTRS_OUT) {
                    ++e;
                } else {
                    push = true;
                    busy = false;
                }
            }
        }
        const uint64_t pushm = __ballot(push);
        if (push)
            pool_store<real>(q, fq + __popcll(pushm & below),
                             (uint32_t)j | ((uint32_t)b << 12) | ((uint32_t)flip << 15) | ((uint32_t)e << 16), n,
                             (int32_t)kk, wu, wv, pp, c);
        fq += __popcll(pushm);
        const bool more = !exhausted || __ballot(busy) != 0ull;
        // flush while a full batch is queued (so the queue holds < 64 entries before the
        // next round adds at most 64), and everything once no new attempts remain
        while (fq >= 64 || (!more && fq > 0)) {
            // 3. final tests of the newest m = min(64, fq) entries. A partial batch (the
            //    day's last tests) spreads each entry over r = 2^lr lanes, r m <= 64: lane jj
            //    of the entry's group takes attempt e + jj of the draw (lane 0 the queued
            //    attempt's final test, the others the next attempts from their own Philox
            //    words), and the first accepted attempt in that order is the draw, exactly
            //    as when they run one after another. Only when all r attempts fail does the
            //    group's last lane go on, from attempt e + r.
            const int m = fq < 64 ? fq : 64;
            const int base = fq - m;
            const int lr = m > 32 ? 0 : (m > 16 ? 1 : (m > 8 ? 2 : (m > 4 ? 3 : (m > 2 ? 4 : (m > 1 ? 5 : 6)))));
            const int r = 1 << lr;
            const int g = lane >> lr, jj = lane & (r - 1);
            const bool mine = g < m;
            uint32_t id2 = 0, wu2 = 0, wv2 = 0;
            int32_t n2 = 0, k2 = 0;
            real p2 = (real)0, spq2 = (real)1, vr2 = (real)0;
            if (mine) {
                const int s = base + g;
                id2 = q->id[s];
                n2 = q->n[s];
                k2 = q->k[s];
                wu2 = q->wu[s];
                wv2 = q->wv[s];
                p2 = q->p[s];
                spq2 = q->spq[s];
                vr2 = q->vr[s];
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            fq = base;
            const int j2 = (int)(id2 & 0xFFFu), b2 = (int)((id2 >> 12) & 7u);
            const bool flip2 = ((id2 >> 15) & 1u) != 0u;
            const DrawStream ds2{(uint32_t)j2, filt, kt, (uint32_t)b2, k0, k1};
            int e2 = (int)(id2 >> 16) + jj;  // this lane's attempt
            int32_t kk2 = k2;
            bool acc = false;
            if (mine) {
                const BtrsConst<real> c2 = btrs_setup_from<real>(n2, p2, spq2, vr2);
                bool need = jj == 0;
                if (jj > 0) {
                    if (e2 >= 256) {
                        acc = true;  // all 256 attempts failed: the mode
                        kk2 = btrs_mode<real>(n2, p2);
                    } else {
                        const W4 w = ds2.call((uint32_t)(e2 >> 1));
                        wu2 = (e2 & 1) ? w.z : w.x;
                        wv2 = (e2 & 1) ? w.w : w.y;
                        const int t = btrs_try<real>(c2, n2, wu2, wv2, kk2);
                        acc = t == BTRS_ACCEPT;
                        need = t == BTRS_FINAL;
                    }
                }
                if (need) acc = btrs_decide<real>(c2, n2, p2, kk2, wu2, wv2);
            }
            // the first accepting lane of each group (g << lr <= lane, so the shift is valid)
            const uint64_t am = __ballot(acc);
            const uint64_t gm = lr == 6 ? am : (am >> (g << lr)) & ((1ull << r) - 1ull);
            const int win = gm ? (g << lr) + (int)__builtin_ctzll(gm) : lane;
            const int32_t kw = __shfl(kk2, win);
            bool push2 = false;
            if (mine) {
                if (gm) {
                    if (jj == 0) flows[b2 * cap + j2] = flip2 ? n2 - kw : kw;
                } else if (jj == r - 1) {
                    const BtrsConst<real> c2 = btrs_setup_from<real>(n2, p2, spq2, vr2);
                    int32_t res = -1;
                    for (++e2;; ++e2) {
                        if (e2 >= 256) {
                            res = btrs_mode<real>(n2, p2);
                            break;
                        }
                        const W4 w = ds2.call((uint32_t)(e2 >> 1));
                        wu2 = (e2 & 1) ? w.z : w.x;
                        wv2 = (e2 & 1) ? w.w : w.y;
                        const int t = btrs_try<real>(c2, n2, wu2, wv2, kk2);
                        if (t == BTRS_OUT) continue;
                        if (t == BTRS_ACCEPT) res = kk2;
                        else push2 = true;
                        break;
                    }
                    if (res >= 0) flows[b2 * cap + j2] = flip2 ? n2 - res : res;
                    id2 = (id2 & 0xFFFFu) | ((uint32_t)e2 << 16);
                }
            }
            const uint64_t pm = __ballot(push2);
            if (push2)
                pool_store<real>(q, fq + __popcll(pm & below), id2, n2, kk2, wu2, wv2, p2,
                                 BtrsConst<real>{spq2, (real)0, (real)0, vr2, (real)0, 0});
            fq += __popcll(pm);
        }
        if (!more && fq == 0) break;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// The day's count update and the per-particle part of log g from the drawn flows. With
// SCORE it adds the day's complete-data score terms from the day-start counts and the
// flows, the same FP64 values in the same order as the per-draw schedule's particle_day.
template <typename real, int MODEL, int OBS, bool SCORE = false>
__device__ __forceinline__ double particle_update(const MConst<real>& mc, int32_t* st, const int32_t* flows,
                                                  int cap, int j, const int32_t* yt, const ScoreDay& sd = ScoreDay{})
{
    if (MODEL == MODEL_SIR) {
        const int32_t nsi = flows[j], nir = flows[cap + j];
        const int32_t S = st[j], I = st[cap + j];
        const int32_t I1 = I + nsi - nir;
        st[j] = S - nsi;
        st[cap + j] = I1;
        if constexpr (SCORE) {
            const real p_si = leave_prob<real>(mc.cinf * (real)I);
            lds_add_f64(sd.sw, cap, j, flow_score<real>(S, p_si, nsi) * ((double)I / sd.n_pop));
            lds_add_f64(sd.sw + 2 * cap, cap, j, flow_score<real>(I, mc.p_ir, nir));
        }
        return obs_part<OBS>(yt[0], OBS == OBS_POIS_PREV ? I1 : nsi, mc.r);
    } else {
        const int32_t nse = flows[j], nei = flows[cap + j], nir = flows[2 * cap + j];
        const int32_t S = st[j], E = st[cap + j], I = st[2 * cap + j];
        const int32_t I1 = I + nei - nir;
        st[j] = S - nse;
        st[cap + j] = E + nse - nei;
        st[2 * cap + j] = I1;
        if constexpr (SCORE) {
            const real p_se = leave_prob<real>(mc.cinf * (real)I);
            lds_add_f64(sd.sw, cap, j, flow_score<real>(S, p_se, nse) * ((double)I / sd.n_pop));
            lds_add_f64(sd.sw + 2 * cap, cap, j, flow_score<real>(E, mc.p_ei, nei));
            lds_add_f64(sd.sw + 4 * cap, cap, j, flow_score<real>(I, mc.p_ir, nir));
            if (sd.nr && nei > 0) {
                const double mu = (double)nei, r = mc.r;
                lds_add_f64(sd.sw + 8 * cap, cap, j, (sd.dpsi - log1p(mu / r)) + (mu - (double)yt[0]) / (r + mu));
            }
        }
        return obs_part<OBS>(yt[0], OBS == OBS_POIS_PREV ? I1 : nei, mc.r);
    }
}

// Multinomial resampling (the paper's particle filter): slot m draws its own uniform
// U_m = floor(x64_m Q / 2^64), x64_m the 64-bit word m & 1 of the Philox call
// (m >> 1, filter, k<<16 | t, 2<<24 | 1<<16), and takes the first j whose inclusive scan
// C_j (in LDS) exceeds it: ancestor j with probability q_j / Q, independently per slot.
__device__ __forceinline__ void multinomial_ancestors(const uint64_t* C, int n, uint64_t Q, uint32_t filt,
                                                      uint32_t kt, uint32_t k0, uint32_t k1, int32_t* anc)
{
    for (int m = (int)threadIdx.x; m < n; m += (int)blockDim.x) {
        const W4 w = philox10((uint32_t)(m >> 1), filt, kt, (S_PF_RS << 24) | (1u << 16), k0, k1);
        const uint64_t x64 = (m & 1) ? ((uint64_t)w.z | ((uint64_t)w.w << 32)) : ((uint64_t)w.x | ((uint64_t)w.y << 32));
        const uint64_t U = __umul64hi(x64, Q);
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (C[mid] > U) hi = mid;
            else lo = mid + 1;
        }
        anc[m] = lo;
    }
}

// LDS layout of one filter (cap = particles rounded up to the block size):
//   C   u64[cap]     quantised weights, then their inclusive scan (then two gather staging rows)
//   tmp i32[cap]     gather staging
//   anc i32[cap]     ancestors            (C, tmp, anc hold the flows while drawing)
//   red RedLds       reduction slots
//   cst f64[T]       per-day observation constants
//   dps f64[T]       per-day psi(y_t + r) - psi(r)  (score launches of SEIR only)
//   lw  real[cap]    log-weights (relative to the last maximum)
//   st  i32[NC*cap]  compartment counts
//   sw  i32[2*NS*cap] score words (score launches only)
//   pool WavePool[blockDim / 64]   (pooled schedules only)
// Issue priority of this wave from the filter's remaining work r (remaining days x N_x,
// as a fraction of the launch's largest filter). The filters resident on a CU each put
// one wave on every SIMD, and the SIMD issues from its oldest wave first: without this,
// the last of four co-resident filters finished about 1.75 times later than the first,
// and the SIMDs spent the tail of the launch with ever fewer waves to hide latency in.
// With the priority falling as the work runs out, the filters that are behind catch up
// and the resident filters finish close together. The levels are fixed points of r; the
// cut points 0.6, 0.3, 0.1 were the fastest of the sets measured (quarters, thirds,
// 0.5/0.2/0.05). Results do not depend on it: it only orders instruction issue.
__device__ __forceinline__ void wave_priority(float r)
{
    if (r > 0.6f) __builtin_amdgcn_s_setprio(3);
    else if (r > 0.3f) __builtin_amdgcn_s_setprio(2);
    else if (r > 0.1f) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

template <typename real, int MODEL, int OBS, int SCHED>
__device__ __attribute__((always_inline)) inline void pf_filter(const PFArgs& a, int item)
{
    constexpr int NC = ModelShape<MODEL>::NC;
    constexpr int NG = ModelShape<MODEL>::NG;
    constexpr bool SCORE = SCHED == PF_SCHED_SCORE || SCHED == PF_SCHED_SCORE_POOLED;
    constexpr bool POOLED = (SCHED == PF_SCHED_POOLED || SCHED == PF_SCHED_SCORE_POOLED) &&
                            (MODEL == MODEL_SIR || MODEL == MODEL_SEIR);
    constexpr int NS = SCORE ? ScoreDims<MODEL>::NS : 0;  // score columns (FP64, two words each)
    const int g = a.items ? a.items[item] : item;
    const int tid = (int)threadIdx.x;
    const int nthr = (int)blockDim.x;
    if (a.active && !a.active[g]) {
        if (first_wave()) {
            a.ll[g] = -INFINITY;
            if constexpr (SCORE)
                for (int d = lane_id(); d < a.D; d += 64) a.score[(size_t)g * a.D + d] = 0.0;
        }
        return;
    }
    const int run_i = g / a.N;
    const uint32_t filt = (uint32_t)(g - run_i * a.N);
    const RunDev run = a.runs[run_i];
    const int T = run.T, nx = run.nx;
    const uint32_t kit = a.k_dev ? (uint32_t)(*a.k_dev) : a.k_const;
    const int cap = ((nx + nthr - 1) / nthr) * nthr;

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int wg_next;  // next draw item of the day (pooled schedule)
    uint64_t* C = reinterpret_cast<uint64_t*>(smem);
    int32_t* tmp = reinterpret_cast<int32_t*>(C + cap);
    int32_t* anc = tmp + cap;
    int32_t* flows = reinterpret_cast<int32_t*>(C);
    RedLds* red = reinterpret_cast<RedLds*>(anc + cap);
    double* cst = reinterpret_cast<double*>(red + 1);
    // score launches of SEIR: each day's psi(y_t + r) - psi(r) after the day constants
    constexpr bool DPSI = SCORE && MODEL == MODEL_SEIR;
    double* dps = cst + T;
    real* lw = reinterpret_cast<real*>(cst + (DPSI ? 2 * T : T));
    int32_t* st = reinterpret_cast<int32_t*>(lw + cap);
    int32_t* sw = st + NC * cap;  // score words (NS columns of two words)
    // offset from the LDS base (not an integer round trip, which would lose the address
    // space and turn every queue access into a generic FLAT access)
    const size_t pool_off = ((size_t)(reinterpret_cast<unsigned char*>(sw + 2 * NS * cap) - smem) + 15) & ~(size_t)15;
    WavePool<real>* pool = reinterpret_cast<WavePool<real>*>(smem + pool_off) + wave_id();

    const double* th = a.theta + (size_t)g * a.D;
    MConst<real> mc;
    model_setup<real, MODEL>(a, th, mc);
    const int32_t* y = a.y + run.y_off;
    for (int t = tid; t < T; t += nthr) {
        double c = 0.0;
        if constexpr (MODEL == MODEL_LG) {
            c = -log(mc.sr) - 0.5 * log(6.283185307179586);
        } else {
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) c = c + obs_const(OBS, y[t * NG + gi], mc.r);
        }
        cst[t] = c;
        if constexpr (DPSI)
            dps[t] = a.D >= 5 ? digamma_f64((double)y[t] + mc.r) - digamma_f64(mc.r) : 0.0;
    }
    for (int j = tid; j < nx; j += nthr) {
        if constexpr (MODEL == MODEL_LG) {
            const double x0 = mc.m0 + mc.s0 * normal_key((uint32_t)j, filt, kit << 16, S_LG << 24, run.k0, run.k1);
            st[j] = __double2loint(x0);
            st[cap + j] = __double2hiint(x0);
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) st[c * cap + j] = mc.x0[c];
        }
#pragma unroll
        for (int c = 0; c < 2 * NS; ++c) sw[c * cap + j] = 0;
        lw[j] = (real)0;
    }
    if (tid == 0) wg_next = 0;
    __syncthreads();

    double ll = 0.0;
    double sl_last = 0.0;  // the last day's FP64 weight sum (the score's normaliser)
    int days = T;  // days run: T, or the day every weight vanished
    const double log_nx = log((double)nx);
    double log_prev = log_nx;  // log of the previous day's weight sum (N_x after a resampling)
    for (int t = 1; t <= T; ++t) {
        const uint32_t kt = (kit << 16) | (uint32_t)t;
        if (a.prio_scale > 0.f) wave_priority((float)(T - t + 1) * (float)nx * a.prio_scale);
        const int32_t* yt = y + (size_t)(t - 1) * NG;
        // 1. propagate and weight: lw[j] <- a_j = lw_j + log g(y_t | x_t^j)
        real amax = (real)-INFINITY;
        ScoreDay sd{};
        if constexpr (SCORE) sd = ScoreDay{sw, a.n_pop, DPSI ? dps[t - 1] : 0.0, MODEL == MODEL_SEIR && a.D >= 5};
        if constexpr (POOLED) {
            draws_pooled<real, MODEL>(mc, st, flows, cap, nx, pool, filt, kt, run.k0, run.k1, &wg_next);
            __syncthreads();  // any wave may have drawn any particle's flows
            if (tid == 0) wg_next = 0;  // for the next day (read again only after further barriers)
            for (int j = tid; j < nx; j += nthr) {
                const double lg = particle_update<real, MODEL, OBS, SCORE>(mc, st, flows, cap, j, yt, sd);
                const real av = lw[j] + (real)lg;
                lw[j] = av;
                amax = av > amax ? av : amax;
            }
        } else {
            // without the filter-level priority, each wave's from its progress through the day;
            // not in score launches, whose two filters per CU ran 4% slower with it over 4096
            // filters (1% faster over 40960; the plain per-draw launch at four filters per CU
            // ran 3-5% faster, one per CU 6-7%)
            constexpr int G = DrawGroups<MODEL>::G;
            const int ptotal = (SCORE || a.prio_scale > 0.f) ? 0 : (cap / nthr) * G;
            for (int j = tid, pass = 0; j < nx; j += nthr, ++pass) {
                const double lg = particle_day<real, MODEL, OBS, SCORE>(
                    mc, st, cap, j, DrawStream{(uint32_t)j, filt, kt, 0u, run.k0, run.k1}, yt, sd, pass * G,
                    ptotal);
                const real av = lw[j] + (real)lg;
                lw[j] = av;
                amax = av > amax ? av : amax;
            }
        }
        if (a.trace_state) {
            for (int j = tid; j < nx; j += nthr)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    a.trace_state[(((size_t)g * T + (t - 1)) * NC + c) * nx + j] = st[c * cap + j];
        }
        const real m = uniform_real<real>(block_max<real>(amax, red));
        if (m == (real)-INFINITY) {
            ll = -INFINITY;
            days = t;
            if (a.trace_inc && first_wave()) {
                for (int tt = t; tt <= T; ++tt) {
                    a.trace_inc[(size_t)g * T + tt - 1] = tt == t ? -INFINITY : 0.0;
                    a.trace_rs[(size_t)g * T + tt - 1] = 0;
                }
            }
            break;
        }
        // 2. normalise by the maximum; FP64 sum and quantised weights. At step s wave w
        //    holds the 64 consecutive particles of chunk s W + w; each chunk is summed by
        //    a wave butterfly and the chunk sums in chunk order, so the sum (and the
        //    likelihood) does not depend on the workgroup size.
        uint64_t q1 = 0, q2 = 0;
        const int nwv = nthr >> 6;
        for (int j = tid, step = 0; j < cap; j += nthr, ++step) {
            double w = 0.0;
            if (j < nx) {
                const real av = lw[j];
                w = exp((double)av - (double)m);
                // w <= 1 (av <= m): q = floor(w 2^32) is 2^32 at w = 1 and fits 32 bits
                // otherwise, where the truncating conversion is the floor; h < 2^25
                const uint64_t q = w >= 1.0 ? (1ull << 32) : (uint64_t)(uint32_t)(w * 4294967296.0);
                // the last day never resamples: score launches keep its FP64 weights instead
                if (SCORE && t == T) reinterpret_cast<double*>(C)[j] = w;
                else C[j] = q;
                const uint32_t h = (uint32_t)(q >> 8);
                q1 += h;
                q2 += (uint64_t)h * h;
                lw[j] = av - m;
            }
            const double cs = wave_sum(w);
            if (lane_id() == 0) red->chunk[step * nwv + wave_id()] = cs;
        }
        double sl = 0.0;
        block_sum3(sl, q1, q2, red);
        sl = 0.0;
        for (int c = 0; c < (cap >> 6); ++c) sl += red->chunk[c];
        sl_last = sl;
        const double lsl = log(sl);
        const double inc = (((double)m + lsl) - log_prev) + cst[t - 1];
        ll = ll + inc;
        log_prev = lsl;
        // 3. resample when ESS < N_x / 2 (never after the last observation)
        const bool rs = uniform_bool(t < T && (a.pf_always || ess_below_half(q1, q2, nx)));
        if (a.trace_inc && first_wave()) {
            a.trace_inc[(size_t)g * T + t - 1] = inc;
            a.trace_rs[(size_t)g * T + t - 1] = rs ? 1 : 0;
        }
        if (rs) {
            const uint64_t Q = block_scan_lds(C, nx, red);
            if (a.multinomial) {
                multinomial_ancestors(C, nx, Q, filt, kt, run.k0, run.k1, anc);
            } else {
                const W4 wd = philox10(0u, filt, kt, S_PF_RS << 24, run.k0, run.k1);
                block_ancestors(C, nx, Q, (uint64_t)wd.x | ((uint64_t)wd.y << 32), anc);
            }
            __syncthreads();
            if (a.trace_anc)
                for (int j = tid; j < nx; j += nthr) a.trace_anc[((size_t)g * T + (t - 1)) * nx + j] = anc[j];
            // the ancestors' words (counts, then the score words), three at a time through the
            // staging rows: tmp and the weights' row C, free once the ancestors are drawn. A
            // barrier separates each group's reads from its writes; each thread touches only
            // its own staging slots, so the next group needs none before it
            constexpr int NW = NC + 2 * NS;
            int32_t* stage = reinterpret_cast<int32_t*>(C);
#pragma unroll
            for (int c0 = 0; c0 < NW; c0 += 3) {
                for (int j = tid; j < nx; j += nthr) {
                    const int aj = anc[j];
                    tmp[j] = st[c0 * cap + aj];
                    if (c0 + 1 < NW) stage[j] = st[(c0 + 1) * cap + aj];
                    if (c0 + 2 < NW) stage[cap + j] = st[(c0 + 2) * cap + aj];
                }
                __syncthreads();
                for (int j = tid; j < nx; j += nthr) {
                    st[c0 * cap + j] = tmp[j];
                    if (c0 + 1 < NW) st[(c0 + 1) * cap + j] = stage[j];
                    if (c0 + 2 < NW) st[(c0 + 2) * cap + j] = stage[cap + j];
                }
            }
            for (int j = tid; j < nx; j += nthr) lw[j] = (real)0;
            log_prev = log_nx;
            // the next day's draws read any particle's counts (the pooled schedule hands
            // out items workgroup-wide): every gathered count must be in place first
            __syncthreads();
        } else if (a.trace_anc) {
            for (int j = tid; j < nx; j += nthr) a.trace_anc[((size_t)g * T + (t - 1)) * nx + j] = j;
        }
    }
    if constexpr (SCORE) {
        // the estimate sum_j w_j s_j / sum_j w_j with the last day's FP64 weights (kept in C),
        // summed per 64-particle chunk and the chunks in order, like the weight sum. The
        // chunk slots still hold the last day's weight sums, which every thread has read
        // only once all have passed this barrier.
        __syncthreads();
        const double* wT = reinterpret_cast<const double*>(C);
        const int nwv = nthr >> 6;
        const bool alive = uniform_bool(ll != -INFINITY);
        for (int d = 0; d < a.D; ++d) {
            double num = 0.0;
            if (alive && d < NS) {
                for (int j = tid, step = 0; j < cap; j += nthr, ++step) {
                    const double v = j < nx ? wT[j] * lds_f64(sw + 2 * d * cap, cap, j) : 0.0;
                    const double cs = wave_sum(v);
                    if (lane_id() == 0) red->chunk[step * nwv + wave_id()] = cs;
                }
                __syncthreads();
                for (int c = 0; c < (cap >> 6); ++c) num += red->chunk[c];
                __syncthreads();  // the chunk slots are reused by the next coordinate
            }
            if (tid == 0) a.score[(size_t)g * a.D + d] = alive ? num / sl_last : 0.0;
        }
    }
    if (first_wave()) a.ll[g] = ll;
    if (a.psteps && tid == 0) atomicAdd(a.psteps + run_i, (unsigned long long)nx * (unsigned long long)days);
}

// One filter per workgroup (a.queue == NULL: filter blockIdx.x), or a persistent grid
// whose workgroups pull the next filter of the work list from an atomic counter until
// the list is exhausted (the list is sorted by cost, longest first).
// Up to 1024 threads (16 waves) per workgroup, which caps the kernel at 128 VGPRs, i.e.
// 4 waves per SIMD: occupancy hides the latency of the FP64 transcendental sequences
// better than a larger register budget. Filters with a large LDS footprint run one
// wide workgroup per CU; small ones run several 256-thread workgroups.
template <typename real, int MODEL, int OBS, int SCHED>
__global__ void __launch_bounds__(1024) k_pf(PFArgs a)
{
    if (!a.queue) {
        if ((int)blockIdx.x < a.n_items) pf_filter<real, MODEL, OBS, SCHED>(a, (int)blockIdx.x);
        return;
    }
    // No branch on the thread index may sit at the top or the bottom of this loop: with
    // one, the compiler moved that lane's work outside a loop the other lanes re-entered
    // through the barrier, and they re-read the old item forever. The first wave fetches
    // (a scalar branch; every lane adds, only lane 0 adds one) and every lane of it stores
    // the same value; pf_filter writes its results the same way.
    __shared__ int next_item;
    for (;;) {
        if (first_wave()) {
            const int got = atomicAdd(a.queue, lane_id() == 0 ? 1 : 0);
            next_item = uniform_i32(got);
        }
        __syncthreads();
        const int item = uniform_i32(next_item);  // scalar: the loop exit is uniform
        __syncthreads();  // every thread has read the item before it is replaced
        if (item >= a.n_items) break;
        pf_filter<real, MODEL, OBS, SCHED>(a, item);
    }
}

// ---------------------------------------------------------------- host side

int pf_score_dims(int model)
{
    if (model == MODEL_SIR) return ScoreDims<MODEL_SIR>::NS;
    if (model == MODEL_SEIR) return ScoreDims<MODEL_SEIR>::NS;
    if (model == MODEL_LG) return ScoreDims<MODEL_LG>::NS;
    return 0;
}

size_t pf_lds_bytes(int model, int prec, int block, int nx, int T, int sched)
{
    int nc = model == MODEL_SIR ? 2 : (model == MODEL_SEIR ? 3 : (model == MODEL_LG ? 2 : 12));
    const size_t cap = (size_t)((nx + block - 1) / block) * block;
    const size_t rb = prec == 0 ? 4 : 8;
    size_t days = (size_t)T;
    if (sched == PF_SCHED_SCORE || sched == PF_SCHED_SCORE_POOLED) {
        nc += 2 * pf_score_dims(model);            // the score words
        if (model == MODEL_SEIR) days += (size_t)T;  // psi(y_t + r) - psi(r) per day
    }
    size_t bytes = cap * 8 + 2 * cap * 4 + sizeof(RedLds) + days * 8 + cap * rb + (size_t)nc * cap * 4;
    if (sched == PF_SCHED_POOLED || sched == PF_SCHED_SCORE_POOLED) {
        const size_t pool = prec == 0 ? sizeof(WavePool<float>) : sizeof(WavePool<double>);
        bytes = ((bytes + 15) & ~(size_t)15) + (size_t)(block / 64) * pool;
    }
    return bytes;
}

int pf_default_block(int model, int prec, int nx, int T, int requested_sched, bool score)
{
    // the workgroup size that keeps the most waves resident per CU (LDS allowing,
    // at most 16 at 128 VGPRs), preferring the pooled schedule by its measured gain
    const int full = ((nx + 63) / 64) * 64;
    int best = full < 256 ? full : 256;
    double best_score = -1.0;
    for (int b = best; b <= 1024; b *= 2) {
        const int sc = pf_pick_schedule(model, prec, b, nx, T, requested_sched, score);
        if (sc < 0) continue;
        const size_t lds = pf_lds_bytes(model, prec, b, nx, T, sc);
        if (lds > PF_LDS_MAX) continue;
        const int per_cu = (int)(PF_LDS_MAX / (lds ? lds : 1));
        int waves = per_cu * (b / 64);
        waves = waves > 16 ? 16 : waves;
        const double merit = waves * (sc == PF_SCHED_POOLED || sc == PF_SCHED_SCORE_POOLED ? 1.4 : 1.0);
        if (merit > best_score + 1e-9) {
            best_score = merit;
            best = b;
        }
        if (b >= full) break;
    }
    return best;
}

int pf_pick_schedule(int model, int prec, int block, int nx, int T, int requested, bool score)
{
    if (score) {
        if (pf_score_dims(model) == 0) return -1;
        const bool ok = (model == MODEL_SIR || model == MODEL_SEIR) &&
                        pf_lds_bytes(model, prec, block, nx, T, PF_SCHED_SCORE_POOLED) <= PF_LDS_MAX;
        // automatic: the per-draw form. The pooled one's extra LDS (the wave pools beside
        // the score words) leaves fewer workgroups per CU, and it measured slower at the
        // SEIR shapes (3.43 against 4.13 ms at N_x = 512, 43.7 against 52.3 ms at N_x =
        // 1024); it is faster for small launch-bound filters, where the autotuner finds it
        if (requested == PF_SCHED_POOLED) return ok ? PF_SCHED_SCORE_POOLED : -1;
        return PF_SCHED_SCORE;
    }
    const bool pooled_ok = (model == MODEL_SIR || model == MODEL_SEIR) &&
                           pf_lds_bytes(model, prec, block, nx, T, PF_SCHED_POOLED) <= PF_LDS_MAX;
    if (requested == PF_SCHED_PER_DRAW) return PF_SCHED_PER_DRAW;
    if (requested == PF_SCHED_POOLED) return pooled_ok ? PF_SCHED_POOLED : -1;
    return pooled_ok ? PF_SCHED_POOLED : PF_SCHED_PER_DRAW;
}

template <typename real, int MODEL, int OBS, int SCHED>
static hipError_t launch_one(int block, size_t lds, const PFArgs& a, hipStream_t s, int grid)
{
    const unsigned g = (unsigned)(a.queue ? grid : a.n_items);
    hipLaunchKernelGGL((k_pf<real, MODEL, OBS, SCHED>), dim3(g), dim3((unsigned)block), lds, s, a);
    return hipGetLastError();
}

template <typename real, int MODEL, int OBS, int SCHED> static const void* kernel_ptr()
{
    return reinterpret_cast<const void*>(&k_pf<real, MODEL, OBS, SCHED>);
}

template <typename real, int SCHED>
static hipError_t launch_model(int model, int obs, int block, size_t lds, const PFArgs& a, hipStream_t s, int grid)
{
    if (model == MODEL_SIR && obs == OBS_POIS_PREV)
        return launch_one<real, MODEL_SIR, OBS_POIS_PREV, SCHED>(block, lds, a, s, grid);
    if (model == MODEL_SIR && obs == OBS_POIS_INC)
        return launch_one<real, MODEL_SIR, OBS_POIS_INC, SCHED>(block, lds, a, s, grid);
    if (model == MODEL_SEIR && obs == OBS_NB_INC)
        return launch_one<real, MODEL_SEIR, OBS_NB_INC, SCHED>(block, lds, a, s, grid);
    if (model == MODEL_AGE && obs == OBS_NB_INC && SCHED == PF_SCHED_PER_DRAW)
        return launch_one<real, MODEL_AGE, OBS_NB_INC, PF_SCHED_PER_DRAW>(block, lds, a, s, grid);
    if constexpr (std::is_same<real, double>::value && (SCHED == PF_SCHED_PER_DRAW || SCHED == PF_SCHED_SCORE))
        if (model == MODEL_LG && obs == OBS_GAUSS)
            return launch_one<double, MODEL_LG, OBS_GAUSS, SCHED>(block, lds, a, s, grid);
    return hipErrorInvalidValue;
}

template <typename real, int SCHED> static const void* kernel_of(int model, int obs)
{
    if (model == MODEL_SIR && obs == OBS_POIS_PREV) return kernel_ptr<real, MODEL_SIR, OBS_POIS_PREV, SCHED>();
    if (model == MODEL_SIR && obs == OBS_POIS_INC) return kernel_ptr<real, MODEL_SIR, OBS_POIS_INC, SCHED>();
    if (model == MODEL_SEIR && obs == OBS_NB_INC) return kernel_ptr<real, MODEL_SEIR, OBS_NB_INC, SCHED>();
    if (model == MODEL_AGE && obs == OBS_NB_INC && SCHED == PF_SCHED_PER_DRAW)
        return kernel_ptr<real, MODEL_AGE, OBS_NB_INC, PF_SCHED_PER_DRAW>();
    if constexpr (std::is_same<real, double>::value && (SCHED == PF_SCHED_PER_DRAW || SCHED == PF_SCHED_SCORE))
        if (model == MODEL_LG && obs == OBS_GAUSS) return kernel_ptr<double, MODEL_LG, OBS_GAUSS, SCHED>();
    return nullptr;
}

bool pf_supported(int model, int obs)
{
    return (model == MODEL_SIR && (obs == OBS_POIS_PREV || obs == OBS_POIS_INC)) ||
           (model == MODEL_SEIR && obs == OBS_NB_INC) || (model == MODEL_AGE && obs == OBS_NB_INC) ||
           (model == MODEL_LG && obs == OBS_GAUSS);
}

static const void* kernel_for(int prec, int model, int obs, int sched)
{
    if (sched == PF_SCHED_SCORE_POOLED)
        return prec == 0 ? kernel_of<float, PF_SCHED_SCORE_POOLED>(model, obs)
                         : kernel_of<double, PF_SCHED_SCORE_POOLED>(model, obs);
    if (sched == PF_SCHED_POOLED)
        return prec == 0 ? kernel_of<float, PF_SCHED_POOLED>(model, obs) : kernel_of<double, PF_SCHED_POOLED>(model, obs);
    if (sched == PF_SCHED_SCORE)
        return prec == 0 ? kernel_of<float, PF_SCHED_SCORE>(model, obs) : kernel_of<double, PF_SCHED_SCORE>(model, obs);
    return prec == 0 ? kernel_of<float, PF_SCHED_PER_DRAW>(model, obs) : kernel_of<double, PF_SCHED_PER_DRAW>(model, obs);
}

hipError_t pf_prepare(int prec, int model, int obs, int sched, size_t lds)
{
    const void* f = kernel_for(prec, model, obs, sched);
    if (!f) return hipErrorInvalidValue;
    if (lds <= 65536) return hipSuccess;
    // the attribute belongs to the kernel on the current device, shared by every launch
    // group and context there: only ever raise it to the largest size asked for
    int dev = 0;
    const hipError_t ed = hipGetDevice(&dev);
    if (ed != hipSuccess) return ed;
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, size_t> raised;
    std::lock_guard<std::mutex> lock(mu);
    size_t& cur = raised[{dev, f}];
    if (lds <= cur) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) cur = lds;
    return e;
}

hipError_t launch_pf(int prec, int model, int obs, int sched, int block, size_t lds, const PFArgs& a, hipStream_t s,
                     int grid)
{
    if (a.n_items <= 0) return hipSuccess;
    if (a.queue && grid <= 0) return hipErrorInvalidValue;
    if (sched == PF_SCHED_POOLED) {
        if (prec == 0) return launch_model<float, PF_SCHED_POOLED>(model, obs, block, lds, a, s, grid);
        return launch_model<double, PF_SCHED_POOLED>(model, obs, block, lds, a, s, grid);
    }
    if (sched == PF_SCHED_SCORE) {
        if (!a.score) return hipErrorInvalidValue;
        if (prec == 0) return launch_model<float, PF_SCHED_SCORE>(model, obs, block, lds, a, s, grid);
        return launch_model<double, PF_SCHED_SCORE>(model, obs, block, lds, a, s, grid);
    }
    if (sched == PF_SCHED_SCORE_POOLED) {
        if (!a.score) return hipErrorInvalidValue;
        if (prec == 0) return launch_model<float, PF_SCHED_SCORE_POOLED>(model, obs, block, lds, a, s, grid);
        return launch_model<double, PF_SCHED_SCORE_POOLED>(model, obs, block, lds, a, s, grid);
    }
    if (prec == 0) return launch_model<float, PF_SCHED_PER_DRAW>(model, obs, block, lds, a, s, grid);
    return launch_model<double, PF_SCHED_PER_DRAW>(model, obs, block, lds, a, s, grid);
}

hipError_t pf_occupancy(int prec, int model, int obs, int sched, int block, size_t lds, int* per_cu)
{
    const void* f = kernel_for(prec, model, obs, sched);
    if (!f) return hipErrorInvalidValue;
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, block, lds);
    *per_cu = n;
    return e;
}

}  // namespace smc2
