// block_ops.h — workgroup-level reductions, scans and the integer systematic
// resampling step shared by the particle-filter kernel and its kernel-level test
// entry point. Block sizes are multiples of 64 (wave64), at most 1024 threads.
#pragma once
#include "device_common.h"

namespace smc2 {

// LDS scratch for reductions: one slot per wave (at most 16 waves).
struct RedLds {
    double max_d[16];
    float max_f[16];
    double sum_d[16];
    uint64_t sum_a[16];
    uint64_t sum_b[16];
    uint64_t scan[16];
    double chunk[64];  // per-64-particle partial sums (at most 4096 particles)
};

template <typename real> __device__ __forceinline__ real* red_max_slot(RedLds* r);
template <> __device__ __forceinline__ float* red_max_slot<float>(RedLds* r) { return r->max_f; }
template <> __device__ __forceinline__ double* red_max_slot<double>(RedLds* r) { return r->max_d; }

// Maximum over the block (exact, order-free).
template <typename real> __device__ __forceinline__ real block_max(real v, RedLds* red)
{
    real* slot = red_max_slot<real>(red);
    v = wave_max(v);
    if (lane_id() == 0) slot[wave_id()] = v;
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6);
    real m = slot[0];
    for (int w = 1; w < nw; ++w) m = slot[w] > m ? slot[w] : m;
    return m;
}

// Sums over the block of one double and two u64 values; fixed reduction order
// (butterfly inside each wave, then waves in index order).
__device__ __forceinline__ void block_sum3(double& s, uint64_t& a, uint64_t& b, RedLds* red)
{
    s = wave_sum(s);
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane_id() == 0) {
        red->sum_d[wave_id()] = s;
        red->sum_a[wave_id()] = a;
        red->sum_b[wave_id()] = b;
    }
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6);
    s = red->sum_d[0];
    a = red->sum_a[0];
    b = red->sum_b[0];
    for (int w = 1; w < nw; ++w) {
        s += red->sum_d[w];
        a += red->sum_a[w];
        b += red->sum_b[w];
    }
}

// Exclusive scan over the block (thread order); returns the exclusive prefix and
// the block total.
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t& total, RedLds* red)
{
    const uint64_t incl = wave_incl_scan(v);
    if (lane_id() == 63) red->scan[wave_id()] = incl;
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6), me = wave_id();
    uint64_t off = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        const uint64_t x = red->scan[w];
        off += (w < me) ? x : 0ull;
        tot += x;
    }
    total = tot;
    return off + incl - v;
}

// ESS < n/2 on the quantised weights q' = q >> 8: 2 (sum q')^2 < n sum q'^2, exact.
__device__ __forceinline__ bool ess_below_half(uint64_t s1, uint64_t s2, int n)
{
    const unsigned __int128 lhs = (unsigned __int128)s1 * s1 * 2u;
    const unsigned __int128 rhs = (unsigned __int128)s2 * (uint64_t)n;
    return lhs < rhs;
}

// In-place inclusive scan of the u64 array C[0..n) held in LDS; returns the total.
// Thread t scans the contiguous chunk [t*c, t*c + c) with c = ceil(n / blockDim),
// so the result is the scan in index order whatever the block size. The caller
// must have made C visible to all threads (a barrier) before the call; C is visible
// to all threads on return.
__device__ __forceinline__ uint64_t block_scan_lds(uint64_t* C, int n, RedLds* red)
{
    const int nthr = (int)blockDim.x, tid = (int)threadIdx.x;
    const int chunk = (n + nthr - 1) / nthr;
    const int lo = tid * chunk;
    const int hi = lo + chunk < n ? lo + chunk : n;
    uint64_t acc = 0;
    for (int e = lo; e < hi; ++e) acc += C[e];
    uint64_t total;
    uint64_t off = block_excl_scan(acc, total, red);
    for (int e = lo; e < hi; ++e) {
        off += C[e];
        C[e] = off;
    }
    __syncthreads();
    return total;
}

// Integer systematic resampling (Sec. IV-B, Eq. cdf and ncopies with the ceil
// convention; the redistribution of Alg. 1 becomes a search of every output slot in
// the cumulative sums): with C the inclusive scan of the quantised weights (total
// Q), output slot m takes ancestor min{ j : n C_j > m Q + U }, U = floor(x64 Q / 2^64),
// i.e. the points m + u, u = U/Q in [0,1), fall in [cdf_{j-1}, cdf_j) with
// cdf_j = n C_j / Q. Slots m = tid, tid + blockDim, ... are written to anc[m].
__device__ __forceinline__ void block_ancestors(const uint64_t* C, int n, uint64_t Q, uint64_t x64,
                                                int32_t* anc)
{
    const uint64_t U = __umul64hi(x64, Q);
    const uint64_t nn = (uint64_t)n;
    for (int m = (int)threadIdx.x; m < n; m += (int)blockDim.x) {
        const uint64_t target = (uint64_t)m * Q + U;
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (nn * C[mid] > target) hi = mid;
            else lo = mid + 1;
        }
        anc[m] = lo;
    }
}

}  // namespace smc2
