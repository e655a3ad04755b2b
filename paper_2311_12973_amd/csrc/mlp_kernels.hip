// mlp_kernels.hip — the learned Gaussian proposal: forward, backward, Adam and the
// held-out check on gfx950 matrix cores.
//
// The random-walk proposal of Sec. IV-A (Eq. proposal) is one choice of q; any q
// whose density is evaluated exactly keeps the weights of Eq. l_weights valid. The
// network maps a sample, whitened by the population's weighted mean c and covariance
// Cholesky factor F (u = F^{-1} (phi - c)), to a Gaussian: mean a and lower Cholesky
// factor L (softplus diagonal + 1e-3), and the proposal is phi' = c + F (a + L z); an
// output of a = 0, L = I proposes the population's Gaussian fit. The network is trained
// after every outer update on the weighted population: the loss of a minibatch is the
// mean over its rows of N w_j NLL(u_j | u_i) for a target j and a randomly paired
// input i (two random affine permutations per epoch), minimised with Adam (0.9, 0.999,
// 1e-8) after clipping the gradient's global norm to 100. The next iteration proposes
// with the network only if its mean weighted NLL on a further pairing is finite and
// below the random walk's.
//
// Tiling: a wave owns 16 rows of a 64-row sub-batch. Every matrix product is a chain
// of v_mfma_f32_16x16x16_bf16 (lane l: A row l%16, B column l%16, k = 4(l/16)..+3;
// result rows 4(l/16)..+3, column l%16). Forward and activation gradients are
// row-local per wave; the weight-gradient tiles (dW3 12, dW2 16, dW1 4) are split over
// the four waves with the sub-batch's 64 rows as the reduction dimension.
#include <math.h>

#include "block_ops.h"
#include "mlp_kernels.h"

namespace smc2 {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define MLP_LOG_2PI 1.8378770664093453
constexpr float MLP_EPS = 1e-3f;
constexpr double MLP_CLIP = 100.0;

// LDS row strides, padded so that the 16 rows one MFMA operand reads fall in
// different banks
constexpr int LD16 = 20, LD64 = 68, LD48 = 52;
constexpr int LDT = MLP_SUB + 8;  // transposed BF16 rows
constexpr int LW1 = 24, LWH = MLP_H + 8;  // BF16 weight rows (W1; W2 and W3), padded the same way

__device__ __forceinline__ short f2bf(float f)
{
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (short)(b >> 16);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct MlpW {                    // one network in BF16 (biases FP32)
    short W1[MLP_H * LW1];       // [h][d], d >= D zero
    short W2[MLP_H * LWH];       // [h][g]
    short W3[MLP_PPAD * LWH];    // [p][g], p >= P zero
    float b1[MLP_H], b2[MLP_H], b3[MLP_PPAD];
};

struct MlpAct {                  // one sub-batch of 64 rows (FP32)
    float U[MLP_SUB * LD16];     // inputs u (d >= D zero)
    float H1[MLP_SUB * LD64];
    float H2[MLP_SUB * LD64];
    float O[MLP_SUB * LD48];     // outputs, then d loss / d outputs
    float Z2[MLP_SUB * LD64];    // d loss / d (W2 h1 + b2)
    float Z1[MLP_SUB * LD64];    // d loss / d (W1 u + b1)
    float UT[MLP_SUB * 8];       // targets
    float wr[MLP_SUB];           // row weights of the loss
    // BF16 copies, transposed ([column][row], stride LDT), of the operands of the
    // weight-gradient products: converted once when the value is written
    short TU[16 * LDT];
    short TH1[MLP_H * LDT];
    short TH2[MLP_H * LDT];
    short TO[MLP_PPAD * LDT];
    short TZ2[MLP_H * LDT];
    short TZ1[MLP_H * LDT];
};

// u = F^{-1} (x - c) for the frame (c[D], F[D][D] lower, row-major), as floats
template <int D> __device__ __forceinline__ void mlp_whiten(const double* fr, const double* x, float* u)
{
    double v[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double s = x[a] - fr[a];
#pragma unroll
        for (int b = 0; b < a; ++b) s -= fr[D + a * D + b] * v[b];
        v[a] = s / fr[D + a * D + a];
        u[a] = (float)v[a];
    }
}

// bytes of the forward-only part (W, U, H1, H2, O)
constexpr size_t MLP_LDS_FWD = sizeof(MlpW) + offsetof(MlpAct, Z2);
constexpr size_t MLP_LDS_TRAIN = sizeof(MlpW) + sizeof(MlpAct);

__device__ void mlp_load_weights(int D, const float* w, MlpW* L)
{
    const int P = mlp_nout(D);
    const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
    const float* W1 = w;
    const float* b1 = W1 + MLP_H * D;
    const float* W2 = b1 + MLP_H;
    const float* b2 = W2 + MLP_H * MLP_H;
    const float* W3 = b2 + MLP_H;
    const float* b3 = W3 + P * MLP_H;
    if (nthr == 256) {
        // every load of the thread issued before the first conversion and store
        float v1[4], v2[16], v3[12];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = tid + 256 * e, h = i >> 4, d = i & 15;
            v1[e] = d < D ? W1[h * D + d] : 0.f;
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) v2[e] = W2[tid + 256 * e];
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            const int i = tid + 256 * e;
            v3[e] = (i / MLP_H) < P ? W3[i] : 0.f;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = tid + 256 * e;
            L->W1[(i >> 4) * LW1 + (i & 15)] = f2bf(v1[e]);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = tid + 256 * e;
            L->W2[(i / MLP_H) * LWH + (i % MLP_H)] = f2bf(v2[e]);
        }
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            const int i = tid + 256 * e;
            L->W3[(i / MLP_H) * LWH + (i % MLP_H)] = f2bf(v3[e]);
        }
    } else {
        for (int i = tid; i < MLP_H * 16; i += nthr) {
            const int h = i >> 4, d = i & 15;
            L->W1[h * LW1 + d] = d < D ? f2bf(W1[h * D + d]) : (short)0;
        }
        for (int i = tid; i < MLP_H * MLP_H; i += nthr) L->W2[(i / MLP_H) * LWH + (i % MLP_H)] = f2bf(W2[i]);
        for (int i = tid; i < MLP_PPAD * MLP_H; i += nthr)
            L->W3[(i / MLP_H) * LWH + (i % MLP_H)] = (i / MLP_H) < P ? f2bf(W3[i]) : (short)0;
    }
    for (int i = tid; i < MLP_H; i += nthr) {
        L->b1[i] = b1[i];
        L->b2[i] = b2[i];
    }
    for (int i = tid; i < MLP_PPAD; i += nthr) L->b3[i] = i < P ? b3[i] : 0.f;
}

// gfx950's 16 x 16 x 32 BF16 product: lane l holds row (A) / column (B) l % 16 at
// k = 8 (l / 16) .. + 7; the accumulator layout is that of the 16 x 16 x 16 form. The
// helpers below take k in steps of 32, and a K that leaves 16 over in one 16 x 16 x 16
// step (lane l: k = 4 (l / 16) .. + 3).
typedef short bf16x8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f32x4 mfma_k32(bf16x8s a, bf16x8s b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// acc[t] += A[16 x K] W_t^T for NT output tiles: A rows FP32 (stride lda), rounded to
// BF16 once per k-step and shared by the tiles; W[n][k] BF16 (stride ldw), tile t from
// row 16 t. The tiles' independent chains interleave; each accumulates over k in order.
template <int K, int NT>
__device__ __forceinline__ void mm_a_wt(const float* A, int lda, const short* W, int ldw, f32x4 (&acc)[NT])
{
    const int l = lane_id(), i = l & 15;
#pragma unroll
    for (int k0 = 0; k0 + 32 <= K; k0 += 32) {
        const int kq = (l >> 4) << 3;
        bf16x8s a;
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = f2bf(A[i * lda + k0 + kq + c]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            bf16x8s b;
#pragma unroll
            for (int c = 0; c < 8; ++c) b[c] = W[(t * 16 + i) * ldw + k0 + kq + c];
            acc[t] = mfma_k32(a, b, acc[t]);
        }
    }
    const int kq = (l >> 4) << 2;
#pragma unroll
    for (int k0 = K - K % 32; k0 < K; k0 += 16) {
        bf16x4 a;
#pragma unroll
        for (int c = 0; c < 4; ++c) a[c] = f2bf(A[i * lda + k0 + kq + c]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            bf16x4 b;
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = W[(t * 16 + i) * ldw + k0 + kq + c];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
}

// acc[t] += A[16 x K] W[:, 16 t .. 16 t + 15]: W[k][n] BF16 (stride ldw)
template <int K, int NT>
__device__ __forceinline__ void mm_a_w(const float* A, int lda, const short* W, int ldw, f32x4 (&acc)[NT])
{
    const int l = lane_id(), i = l & 15;
#pragma unroll
    for (int k0 = 0; k0 + 32 <= K; k0 += 32) {
        const int kq = (l >> 4) << 3;
        bf16x8s a;
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = f2bf(A[i * lda + k0 + kq + c]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            bf16x8s b;
#pragma unroll
            for (int c = 0; c < 8; ++c) b[c] = W[(k0 + kq + c) * ldw + t * 16 + i];
            acc[t] = mfma_k32(a, b, acc[t]);
        }
    }
    const int kq = (l >> 4) << 2;
#pragma unroll
    for (int k0 = K - K % 32; k0 < K; k0 += 16) {
        bf16x4 a;
#pragma unroll
        for (int c = 0; c < 4; ++c) a[c] = f2bf(A[i * lda + k0 + kq + c]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            bf16x4 b;
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = W[(k0 + kq + c) * ldw + t * 16 + i];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
}

// acc += X^T Y over the sub-batch's rows, from the transposed BF16 copies XT[m][row] and
// YT[n][row] (stride LDT) of the tile's first output row / column
__device__ __forceinline__ f32x4 mm_t(const short* XT, const short* YT, f32x4 acc)
{
    static_assert(MLP_SUB % 32 == 0, "sub-batch rows in steps of 32");
    const int l = lane_id(), i = l & 15, kq = (l >> 4) << 3;
#pragma unroll
    for (int k0 = 0; k0 < MLP_SUB; k0 += 32) {
        bf16x8s a, b;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            a[c] = XT[i * LDT + k0 + kq + c];
            b[c] = YT[i * LDT + k0 + kq + c];
        }
        acc = mfma_k32(a, b, acc);
    }
    return acc;
}

// tanh from the hardware exponential and reciprocal (a few FP32 units of error, far
// below the BF16 rounding the next layer applies): the odd series through x^7 below
// |x| = 1/16 (truncation < 2e-13 relative), 1 - 2 / (exp(2|x|) + 1) above
__device__ __forceinline__ float tanh_fast(float x)
{
    const float ax = fabsf(x);
    float r;
    if (ax < 0.0625f) {
        const float x2 = x * x;
        r = ax * (1.f + x2 * (-0.333333333f + x2 * (0.133333333f + x2 * -0.0539682540f)));
    } else {
        r = 1.f - 2.f * __builtin_amdgcn_rcpf(__expf(2.f * ax) + 1.f);
    }
    return copysignf(r, x);
}

// forward pass of the wave's 16 rows (from row r0 of the sub-batch); with TRAIN the
// hidden layers also go to their transposed BF16 copies
template <bool TRAIN> __device__ void mlp_fwd16(const MlpW* W, MlpAct* A, int r0)
{
    const int l = lane_id(), j = l & 15, rq = (l >> 4) << 2;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{W->b1[t * 16 + j], W->b1[t * 16 + j], W->b1[t * 16 + j], W->b1[t * 16 + j]};
    mm_a_wt<16, 4>(A->U + r0 * LD16, LD16, W->W1, LW1, acc);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float h = tanh_fast(acc[t][c]);
            A->H1[(r0 + rq + c) * LD64 + t * 16 + j] = h;
            if (TRAIN) A->TH1[(t * 16 + j) * LDT + r0 + rq + c] = f2bf(h);
        }
    wave_sync();
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{W->b2[t * 16 + j], W->b2[t * 16 + j], W->b2[t * 16 + j], W->b2[t * 16 + j]};
    mm_a_wt<MLP_H, 4>(A->H1 + r0 * LD64, LD64, W->W2, LWH, acc);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float h = tanh_fast(acc[t][c]);
            A->H2[(r0 + rq + c) * LD64 + t * 16 + j] = h;
            if (TRAIN) A->TH2[(t * 16 + j) * LDT + r0 + rq + c] = f2bf(h);
        }
    wave_sync();
    f32x4 ao[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) ao[t] = f32x4{W->b3[t * 16 + j], W->b3[t * 16 + j], W->b3[t * 16 + j], W->b3[t * 16 + j]};
    mm_a_wt<MLP_H, 3>(A->H2 + r0 * LD64, LD64, W->W3, LWH, ao);
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) A->O[(r0 + rq + c) * LD48 + t * 16 + j] = ao[t][c];
    wave_sync();
}

// activation gradients of the wave's 16 rows from d loss / d outputs (in A->O), with
// their transposed BF16 copies
__device__ void mlp_bwd16(const MlpW* W, MlpAct* A, int r0)
{
    const int l = lane_id(), j = l & 15, rq = (l >> 4) << 2;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    mm_a_w<MLP_PPAD, 4>(A->O + r0 * LD48, LD48, W->W3, LWH, acc);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int at = (r0 + rq + c) * LD64 + t * 16 + j;
            const float h = A->H2[at];
            const float z = acc[t][c] * (1.f - h * h);
            A->Z2[at] = z;
            A->TZ2[(t * 16 + j) * LDT + r0 + rq + c] = f2bf(z);
        }
    wave_sync();
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    mm_a_w<MLP_H, 4>(A->Z2 + r0 * LD64, LD64, W->W2, LWH, acc);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int at = (r0 + rq + c) * LD64 + t * 16 + j;
            const float h = A->H1[at];
            const float z = acc[t][c] * (1.f - h * h);
            A->Z1[at] = z;
            A->TZ1[(t * 16 + j) * LDT + r0 + rq + c] = f2bf(z);
        }
    wave_sync();
}

// transposed BF16 copy of the output gradients of the wave's 16 rows
__device__ __forceinline__ void mlp_copy_ograd(MlpAct* A, int r0)
{
    const int l = lane_id();
    for (int e = l; e < 16 * MLP_PPAD; e += 64) {
        const int rr = r0 + (e & 15), pp = e >> 4;
        A->TO[pp * LDT + rr] = f2bf(A->O[rr * LD48 + pp]);
    }
    wave_sync();
}

// bias gradients of the wave's 16 rows, added to the lane's partial sums (lane l:
// column l of the output gradients (l < 48), of Z2 and of Z1)
__device__ __forceinline__ void mlp_bias16(const MlpAct* A, int r0, float& b3, float& b2, float& b1)
{
    const int l = lane_id();
    float s3 = 0.f, s2 = 0.f, s1 = 0.f;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        if (l < MLP_PPAD) s3 += A->O[(r0 + rr) * LD48 + l];
        s2 += A->Z2[(r0 + rr) * LD64 + l];
        s1 += A->Z1[(r0 + rr) * LD64 + l];
    }
    b3 += s3;
    b2 += s2;
    b1 += s1;
}

// the four waves' bias partial sums in wave order, into grad[] (parameter layout);
// part is LDS scratch of 4 x 176 floats; every thread of the block calls it
template <int D> __device__ double mlp_bias_write(float* part, float b3, float b2, float b1, float* grad)
{
    constexpr int P = D + D * (D + 1) / 2;
    const int l = lane_id(), w = wave_id(), tid = (int)threadIdx.x;
    if (l < MLP_PPAD) part[w * 176 + l] = b3;
    part[w * 176 + 48 + l] = b2;
    part[w * 176 + 112 + l] = b1;
    __syncthreads();
    double ss = 0.0;  // squares of the entries written (for the gradient norm)
    if (tid < 176) {
        const float s = ((part[tid] + part[176 + tid]) + part[352 + tid]) + part[528 + tid];
        if (tid < 48) {
            if (tid < P) {
                grad[mlp_nparams(D) - P + tid] = s;
                ss = (double)s * (double)s;
            }
        } else if (tid < 112) {
            grad[MLP_H * D + MLP_H + MLP_H * MLP_H + tid - 48] = s;
            ss = (double)s * (double)s;
        } else {
            grad[MLP_H * D + tid - 112] = s;
            ss = (double)s * (double)s;
        }
    }
    __syncthreads();
    return ss;
}

// weight-gradient tiles of the sub-batch accumulated in acc[] (wave w: tiles w + 4q)
__device__ void mlp_wgrad(const MlpAct* A, f32x4 (&acc)[8])
{
    const int w = wave_id();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int t = w + 4 * q;
        if (t < 12) {
            acc[q] = mm_t(A->TO + (t >> 2) * 16 * LDT, A->TH2 + (t & 3) * 16 * LDT, acc[q]);
        } else if (t < 28) {
            acc[q] = mm_t(A->TZ2 + ((t - 12) >> 2) * 16 * LDT, A->TH1 + ((t - 12) & 3) * 16 * LDT, acc[q]);
        } else {
            acc[q] = mm_t(A->TZ1 + (t - 28) * 16 * LDT, A->TU, acc[q]);
        }
    }
}

// adds the tiles to grad[] (parameter layout)
template <int D> __device__ double mlp_scatter_wgrad(const f32x4 (&acc)[8], float* grad)
{
    constexpr int P = D + D * (D + 1) / 2;
    double ss = 0.0;  // squares of the entries written (for the gradient norm)
    float* gW1 = grad;
    float* gW2 = gW1 + MLP_H * D + MLP_H;
    float* gW3 = gW2 + MLP_H * MLP_H + MLP_H;
    const int l = lane_id(), j = l & 15, rq = (l >> 4) << 2, w = wave_id();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int t = w + 4 * q;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = rq + c;
            if (t < 12) {
                const int p = (t >> 2) * 16 + i, g = (t & 3) * 16 + j;
                if (p < P) {
                    gW3[p * MLP_H + g] = acc[q][c];
                    ss += (double)acc[q][c] * (double)acc[q][c];
                }
            } else if (t < 28) {
                const int h = ((t - 12) >> 2) * 16 + i, g = ((t - 12) & 3) * 16 + j;
                gW2[h * MLP_H + g] = acc[q][c];
                ss += (double)acc[q][c] * (double)acc[q][c];
            } else {
                const int h = (t - 28) * 16 + i;
                if (j < D) {
                    gW1[h * D + j] = acc[q][c];
                    ss += (double)acc[q][c] * (double)acc[q][c];
                }
            }
        }
    }
    return ss;
}

// parameter i (layout W1 b1 W2 b2 W3 b3) into the LDS copy of the network
template <int D> __device__ __forceinline__ void mlp_store_weight(MlpW* L, int i, float v)
{
    constexpr int P = D + D * (D + 1) / 2;
    if (i < MLP_H * D) {
        const int h = i / D;
        L->W1[h * LW1 + (i - h * D)] = f2bf(v);
        return;
    }
    i -= MLP_H * D;
    if (i < MLP_H) {
        L->b1[i] = v;
        return;
    }
    i -= MLP_H;
    if (i < MLP_H * MLP_H) {
        L->W2[(i >> 6) * LWH + (i & 63)] = f2bf(v);
        return;
    }
    i -= MLP_H * MLP_H;
    if (i < MLP_H) {
        L->b2[i] = v;
        return;
    }
    i -= MLP_H;
    if (i < P * MLP_H) {
        L->W3[(i >> 6) * LWH + (i & 63)] = f2bf(v);
        return;
    }
    L->b3[i - P * MLP_H] = v;
}

__device__ __forceinline__ float softplus_f(float x) { return x > 30.f ? x : log1pf(expf(x)); }

// NLL of row r (targets A->UT) from its outputs; with grad, replaces the outputs by
// scale * d NLL / d o (padding columns stay zero).
template <int D> __device__ float mlp_row_nll(MlpAct* A, int r, float scale, bool grad)
{
    float* o = A->O + r * LD48;
    const float* ut = A->UT + r * 8;
    float L[D * (D + 1) / 2], v[D], w[D];
    float quad = 0.f, logdet = 0.f;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int jj = 0; jj <= i; ++jj) {
            const float x = o[D + i * (i + 1) / 2 + jj];
            L[i * (i + 1) / 2 + jj] = (i == jj) ? softplus_f(x) + MLP_EPS : x;
        }
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float s = ut[i] - o[i];
#pragma unroll
        for (int jj = 0; jj < i; ++jj) s -= L[i * (i + 1) / 2 + jj] * v[jj];
        v[i] = s / L[i * (i + 1) / 2 + i];
        quad += v[i] * v[i];
        logdet += logf(L[i * (i + 1) / 2 + i]);
    }
    const float nll = 0.5f * quad + logdet + 0.5f * (float)D * (float)MLP_LOG_2PI;
    if (grad) {
#pragma unroll
        for (int i = D - 1; i >= 0; --i) {
            float s = v[i];
#pragma unroll
            for (int jj = i + 1; jj < D; ++jj) s -= L[jj * (jj + 1) / 2 + i] * w[jj];
            w[i] = s / L[i * (i + 1) / 2 + i];
        }
        float od[D];
#pragma unroll
        for (int i = 0; i < D; ++i) od[i] = o[D + i * (i + 1) / 2 + i];
#pragma unroll
        for (int i = 0; i < D; ++i) o[i] = scale * -w[i];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int jj = 0; jj <= i; ++jj) {
                float g = -w[i] * v[jj];
                if (i == jj) g = (g + 1.f / L[i * (i + 1) / 2 + i]) * (1.f / (1.f + expf(-od[i])));
                o[D + i * (i + 1) / 2 + jj] = scale * g;
            }
    }
    return nll;
}

// the random affine permutation of (k, epoch, which): a, b with gcd(a, N) = 1
__device__ __forceinline__ void mlp_perm_dev(uint64_t seed, uint32_t k, uint32_t e, uint32_t which, int N,
                                             uint64_t& a, uint64_t& b)
{
    const W4 x = philox10(k, e, which, S_MLP_PERM << 24, (uint32_t)seed, (uint32_t)(seed >> 32));
    a = 1;
    b = 0;
    if (N > 1) {
        a = 1 + (uint64_t)x.x % (uint64_t)(N - 1);
        for (;;) {
            uint64_t p = a, q = (uint64_t)N;
            while (q) {
                const uint64_t t = p % q;
                p = q;
                q = t;
            }
            if (p == 1) break;
            a = a % (uint64_t)(N - 1) + 1;
        }
        b = (uint64_t)x.y % (uint64_t)N;
    }
}

// Fixed-order block sum of E doubles per thread (butterfly per wave, waves in order);
// every thread gets the totals. lds holds 16 x E doubles.
template <int E> __device__ void mlp_block_sum(double (&v)[E], double* lds)
{
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = wave_sum(v[e]);
    __syncthreads();
    if (lane_id() == 0)
#pragma unroll
        for (int e = 0; e < E; ++e) lds[wave_id() * E + e] = v[e];
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[w * E + e];
        v[e] = s;
    }
}

// ------------------------------------------------------------------ forward over a population
template <int D>
__global__ void __launch_bounds__(256) k_mlp_forward(MlpArrays m, MlpParams p, OuterArrays o)
{
    constexpr int P = D + D * (D + 1) / 2;
    const int r = (int)blockIdx.y;
    const int k = *o.k_dev;
    if (k < 2 || !m.use[r]) return;
    extern __shared__ __align__(16) unsigned char smem[];
    MlpW* W = reinterpret_cast<MlpW*>(smem);
    MlpAct* A = reinterpret_cast<MlpAct*>(smem + sizeof(MlpW));
    const int NP = mlp_nparams(D);
    mlp_load_weights(D, m.params + (size_t)r * NP, W);
    const double* fr = m.frame + (size_t)r * (D + D * D);
    const int row0 = (int)blockIdx.x * MLP_SUB;
    const int tid = (int)threadIdx.x;
    if (tid < MLP_SUB) {
        const int i = row0 + tid;
        float u[16];
#pragma unroll
        for (int d = 0; d < 16; ++d) u[d] = 0.f;
        if (i < p.N) mlp_whiten<D>(fr, o.phi + ((size_t)r * p.N + i) * D, u);
#pragma unroll
        for (int d = 0; d < 16; ++d) A->U[tid * LD16 + d] = u[d];
    }
    __syncthreads();
    mlp_fwd16<false>(W, A, wave_id() * 16);
    __syncthreads();
    for (int e = tid; e < MLP_SUB * P; e += (int)blockDim.x) {
        const int rr = e / P, pp = e - rr * P, i = row0 + rr;
        if (i < p.N) m.out[((size_t)r * p.N + i) * P + pp] = A->O[rr * LD48 + pp];
    }
}

// ------------------------------------------------------------------ training
// Training prologue of run r (every thread of the block): the population's weights
// W = log sum exp (log w), the frame (weighted mean c and the Cholesky factor F of the
// weighted covariance; the diagonal of the standard deviations when a pivot is not above
// 1e-12 of its coordinate's raw second moment) into frs (LDS) and m.frame, and the
// population whitened in that frame with N w_i, read by the sub-batches in their random
// pairing order. A is free LDS scratch here.
template <int D>
__device__ void mlp_train_prologue(const MlpArrays& m, const MlpParams& p, const OuterArrays& o, int r, MlpAct* A,
                                   double* red, double* frs)
{
    const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
    const int N = p.N;
    const double* phi = o.phi + (size_t)r * N * D;
    const double* logw = o.logw + (size_t)r * N;
    // weights of the population: W = log sum exp (log w)
    double mx = -INFINITY;
    for (int i = tid; i < N; i += nthr) mx = logw[i] > mx ? logw[i] : mx;
    {
        RedLds* rl = reinterpret_cast<RedLds*>(A);  // the activation area is free here
        mx = uniform_f64(block_max<double>(mx, rl));
    }
    double sw[1] = {0.0};
    for (int i = tid; i < N; i += nthr) sw[0] += exp(logw[i] - mx);
    mlp_block_sum<1>(sw, red);
    const double LW = mx + log(sw[0]);
    // frame: weighted mean c and the Cholesky factor F of the weighted covariance
    // (diagonal of the standard deviations when a pivot is not above 1e-12 of its
    // coordinate's raw second moment)
    {
        double acc[D];
#pragma unroll
        for (int d = 0; d < D; ++d) acc[d] = 0.0;
        for (int i = tid; i < N; i += nthr) {
            const double wn = exp(logw[i] - LW);
#pragma unroll
            for (int d = 0; d < D; ++d) acc[d] += wn * phi[(size_t)i * D + d];
        }
        mlp_block_sum<D>(acc, red);
        double c[D];
#pragma unroll
        for (int d = 0; d < D; ++d) c[d] = acc[d];
        // covariance rows one at a time (D sums per pass)
        for (int a = 0; a < D; ++a) {
            double cv[D];
#pragma unroll
            for (int b = 0; b < D; ++b) cv[b] = 0.0;
            for (int i = tid; i < N; i += nthr) {
                const double wn = exp(logw[i] - LW);
                const double za = phi[(size_t)i * D + a] - c[a];
#pragma unroll
                for (int b = 0; b < D; ++b) cv[b] += wn * za * (phi[(size_t)i * D + b] - c[b]);
            }
            mlp_block_sum<D>(cv, red);
            if (tid == 0)
#pragma unroll
                for (int b = 0; b < D; ++b) frs[D + a * D + b] = cv[b];  // covariance, factored below
        }
        if (tid == 0) {
            double C[D * D], F[D * D];
#pragma unroll
            for (int e = 0; e < D * D; ++e) {
                C[e] = frs[D + e];
                F[e] = 0.0;
            }
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
#pragma unroll
            for (int d = 0; d < D; ++d) frs[d] = c[d];
#pragma unroll
            for (int e = 0; e < D * D; ++e) frs[D + e] = F[e];
        }
        __syncthreads();
    }
    double* fr_out = m.frame + (size_t)r * (D + D * D);
    for (int d = tid; d < D + D * D; d += nthr) fr_out[d] = frs[d];

    // the population once in the network's frame: whitened rows and N w_i (FP64), read
    // by the sub-batches below in their random pairing order
    float* rows = m.rows + (size_t)r * N * MLP_ROW;
    double* wfull = m.wfull + (size_t)r * N;
    for (int i = tid; i < N; i += nthr) {
        float u[16];
        mlp_whiten<D>(frs, phi + (size_t)i * D, u);
#pragma unroll
        for (int d = 0; d < MLP_ROW; ++d) rows[(size_t)i * MLP_ROW + d] = d < D ? u[d] : 0.f;
        wfull[i] = (double)N * exp(logw[i] - LW);
    }
    __syncthreads();

}

// Held-out check of run r after training: the mean weighted NLL of the network W (LDS)
// on the pairing of "epoch" E against the random walk's; the next iteration proposes
// with the network only if it is finite and lower. mlp_heldout_rows adds the weighted
// NLLs of the pairs of sub-batches s_lo, s_lo + 64, ... below s_hi to the thread's sums
// (threads < 64 hold a row each; every thread of the block calls it); frs holds the
// frame (LDS), A is LDS scratch.
template <int D>
__device__ void mlp_heldout_rows(const MlpArrays& m, const MlpParams& p, const OuterArrays& o, int r, int k,
                                 uint64_t seed, const MlpW* W, MlpAct* A, const double* frs, int s_lo, int s_hi,
                                 double (&sums)[2])
{
    const int tid = (int)threadIdx.x;
    const int N = p.N;
    const double* phi = o.phi + (size_t)r * N * D;
    const float* rows = m.rows + (size_t)r * N * MLP_ROW;
    const double* wfull = m.wfull + (size_t)r * N;
    uint64_t ta, tb, ia, ib;
    mlp_perm_dev(seed, (uint32_t)k, (uint32_t)p.epochs, 0u, N, ta, tb);
    mlp_perm_dev(seed, (uint32_t)k, (uint32_t)p.epochs, 1u, N, ia, ib);
    double sls = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) sls += log(frs[D + d * D + d]);
    for (int s0 = s_lo; s0 < s_hi; s0 += MLP_SUB) {
        int jt = 0, ii = 0;
        double wt = 0.0;
        if (tid < MLP_SUB) {
            const int rr = s0 + tid;
            const bool valid = rr < N;
            jt = valid ? (int)((ta * (uint64_t)rr + tb) % (uint64_t)N) : 0;
            ii = valid ? (int)((ia * (uint64_t)rr + ib) % (uint64_t)N) : 0;
            wt = valid ? wfull[jt] : 0.0;
#pragma unroll
            for (int d = 0; d < 16; ++d)
                A->U[tid * LD16 + d] = (valid && d < MLP_ROW) ? rows[(size_t)ii * MLP_ROW + d] : 0.f;
#pragma unroll
            for (int d = 0; d < 8; ++d) A->UT[tid * 8 + d] = valid ? rows[(size_t)jt * MLP_ROW + d] : 0.f;
        }
        __syncthreads();
        mlp_fwd16<false>(W, A, wave_id() * 16);
        __syncthreads();
        if (tid < MLP_SUB && wt > 0.0) {
            const float nll = mlp_row_nll<D>(A, tid, 0.f, false);
            sums[0] += wt * ((double)nll + sls);
            // random walk: -log N(phi_j; phi_i, L L^T)
            double v[D], quad = 0.0, ld = 0.0;
#pragma unroll
            for (int a2 = 0; a2 < D; ++a2) {
                double sa = phi[(size_t)jt * D + a2] - phi[(size_t)ii * D + a2];
#pragma unroll
                for (int b2 = 0; b2 < a2; ++b2) sa -= p.lrw[a2 * D + b2] * v[b2];
                v[a2] = sa / p.lrw[a2 * D + a2];
                quad += v[a2] * v[a2];
                ld += log(p.lrw[a2 * D + a2]);
            }
            sums[1] += wt * (0.5 * quad + ld + 0.5 * D * MLP_LOG_2PI);
        }
        __syncthreads();
    }
}

// the decision from the summed weighted NLLs (one thread)
__device__ __forceinline__ void mlp_heldout_decide(const MlpArrays& m, const MlpParams& p, const OuterArrays& o,
                                                   int r, int k, double sm, double sr)
{
    const double nm = sm / p.N, nr = sr / p.N;
    m.score[2 * r] = nm;
    m.score[2 * r + 1] = nr;
    m.use[r] = (isfinite(nm) && nm < nr) ? 1 : 0;
    o.records[((size_t)r * p.K + (k - 1)) * p.rec_len + p.rec_len - 1] = nm - nr;
}

template <int D>
__device__ void mlp_heldout(const MlpArrays& m, const MlpParams& p, const OuterArrays& o, int r, int k,
                            uint64_t seed, const MlpW* W, MlpAct* A, double* red, const double* frs)
{
    double sums[2] = {0.0, 0.0};
    mlp_heldout_rows<D>(m, p, o, r, k, seed, W, A, frs, 0, p.N, sums);
    mlp_block_sum<2>(sums, red);
    if (threadIdx.x == 0) mlp_heldout_decide(m, p, o, r, k, sums[0], sums[1]);
}

template <int D>
__global__ void __launch_bounds__(256) k_mlp_train(MlpArrays m, MlpParams p, OuterArrays o, const uint64_t* seeds)
{
    const int r = (int)blockIdx.x;
    const int tid = (int)threadIdx.x;
    const int N = p.N;
    const int k = *o.k_dev;
    if (o.status[r] != 0) return;  // every weight vanished: nothing to learn from
    extern __shared__ __align__(16) unsigned char smem[];
    MlpW* W = reinterpret_cast<MlpW*>(smem);
    MlpAct* A = reinterpret_cast<MlpAct*>(smem + sizeof(MlpW));
    __shared__ double red[16 * (2 * DMAX + 1)];
    __shared__ double frs[DMAX + DMAX * DMAX];
    const int NP = mlp_nparams(D);
    float* prm = m.params + (size_t)r * NP;
    float* am = m.adam_m + (size_t)r * NP;
    float* av = m.adam_v + (size_t)r * NP;
    float* grad = m.grad + (size_t)r * NP;
    const uint64_t seed = seeds[r];

    mlp_train_prologue<D>(m, p, o, r, A, red, frs);
    const float* rows = m.rows + (size_t)r * N * MLP_ROW;
    const double* wfull = m.wfull + (size_t)r * N;

    const int B = (p.batch < 1 || p.batch > N) ? N : p.batch;
    int t_adam = m.adam_t[r];
    mlp_load_weights(D, prm, W);
    __syncthreads();
    for (int ep = 0; ep < p.epochs; ++ep) {
        uint64_t ta, tb, ia, ib;
        mlp_perm_dev(seed, (uint32_t)k, (uint32_t)ep, 0u, N, ta, tb);
        mlp_perm_dev(seed, (uint32_t)k, (uint32_t)ep, 1u, N, ia, ib);
        // rows of sub-batch (b0, s0) of a minibatch of nb rows (threads < MLP_SUB)
        auto fetch = [&](int b0, int s0, int nb, float* fu, float* ft, float& fw) {
            const int rr = b0 + s0 + tid;
#pragma unroll
            for (int d = 0; d < MLP_ROW; ++d) fu[d] = ft[d] = 0.f;
            fw = 0.f;
            if (s0 + tid < nb) {
                const int jt = (int)((ta * (uint64_t)rr + tb) % (uint64_t)N);
                const int ii = (int)((ia * (uint64_t)rr + ib) % (uint64_t)N);
#pragma unroll
                for (int d = 0; d < MLP_ROW; ++d) {
                    fu[d] = rows[(size_t)ii * MLP_ROW + d];
                    ft[d] = rows[(size_t)jt * MLP_ROW + d];
                }
                fw = (float)(wfull[jt] / (double)nb);
            }
        };
        for (int b0 = 0; b0 < N; b0 += B) {
            const int nb = (N - b0) < B ? (N - b0) : B;
            f32x4 acc[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
            float bb3 = 0.f, bb2 = 0.f, bb1 = 0.f;  // bias-gradient partial sums of this wave's rows
            float cu[MLP_ROW], ct[MLP_ROW], cw = 0.f;  // the next sub-batch's rows (threads < MLP_SUB)
            if (tid < MLP_SUB) fetch(b0, 0, nb, cu, ct, cw);
            for (int s0 = 0; s0 < nb; s0 += MLP_SUB) {
                // rows of the sub-batch, then the loads of the following one, which
                // complete while this one is computed
                if (tid < MLP_SUB) {
#pragma unroll
                    for (int d = 0; d < 16; ++d) {
                        const float ud = d < MLP_ROW ? cu[d] : 0.f;
                        A->U[tid * LD16 + d] = ud;
                        A->TU[d * LDT + tid] = f2bf(ud);
                    }
#pragma unroll
                    for (int d = 0; d < 8; ++d) A->UT[tid * 8 + d] = ct[d];
                    A->wr[tid] = cw;
                    if (s0 + MLP_SUB < nb) fetch(b0, s0 + MLP_SUB, nb, cu, ct, cw);
                }
                __syncthreads();
                mlp_fwd16<true>(W, A, wave_id() * 16);
                if (lane_id() < 16) mlp_row_nll<D>(A, wave_id() * 16 + lane_id(), A->wr[wave_id() * 16 + lane_id()], true);
                wave_sync();
                mlp_copy_ograd(A, wave_id() * 16);
                mlp_bwd16(W, A, wave_id() * 16);
                mlp_bias16(A, wave_id() * 16, bb3, bb2, bb1);
                __syncthreads();
                mlp_wgrad(A, acc);
                __syncthreads();  // the next sub-batch overwrites the activations
            }
            // minibatch gradient in parameter layout; its squared norm from the values
            // as they are written
            double nn[1] = {mlp_scatter_wgrad<D>(acc, grad)};
            nn[0] += mlp_bias_write<D>(A->H1, bb3, bb2, bb1, grad);
            mlp_block_sum<1>(nn, red);
            const double nrm = sqrt(nn[0]);
            const double clip = nrm > MLP_CLIP ? MLP_CLIP / nrm : 1.0;
            ++t_adam;
            const float c1 = 1.f - powf(0.9f, (float)t_adam), c2 = 1.f - powf(0.999f, (float)t_adam);
            // Adam, each updated weight also written to the network's LDS copy: the
            // thread's parameters i = tid + 256 e in chunks of 8 whose loads are all
            // issued before the first update, so they overlap
            {
                constexpr int PER = (mlp_np_const(D) + 255) / 256, CH = 8;
#pragma nounroll
                for (int e0 = 0; e0 < PER; e0 += CH) {
                    float g[CH], mo[CH], vo[CH], po[CH];
#pragma unroll
                    for (int e = 0; e < CH; ++e) {
                        const int i = tid + 256 * (e0 + e);
                        if (e0 + e < PER && i < NP) {
                            g[e] = grad[i];
                            mo[e] = am[i];
                            vo[e] = av[i];
                            po[e] = prm[i];
                        }
                    }
#pragma unroll
                    for (int e = 0; e < CH; ++e) {
                        const int i = tid + 256 * (e0 + e);
                        if (e0 + e < PER && i < NP) {
                            const float gi = (float)((double)g[e] * clip);
                            const float mi = 0.9f * mo[e] + 0.1f * gi;
                            const float vi = 0.999f * vo[e] + 0.001f * gi * gi;
                            const float pn = po[e] - p.lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
                            am[i] = mi;
                            av[i] = vi;
                            prm[i] = pn;
                            mlp_store_weight<D>(W, i, pn);
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    if (tid == 0) m.adam_t[r] = t_adam;

    mlp_heldout<D>(m, p, o, r, k, seed, W, A, red, frs);
}

// ------------------------------------------------------------------ kernel-level entry points
// ------------------------------------------------------------------ split training
// The same training with a minibatch's sub-batches spread over workgroups, for few
// runs (one workgroup per run would leave most CUs idle): per minibatch one launch
// computes each sub-batch's gradient in its own workgroup (the network loaded from the
// master weights), and a second sums them in sub-batch order and takes the clipped
// Adam step. The sums group the rows differently from one workgroup's running
// accumulation, so the two forms agree to FP32 rounding, not bit for bit.

template <int D>
__global__ void __launch_bounds__(256) k_mlp_prep(MlpArrays m, MlpParams p, OuterArrays o)
{
    const int r = (int)blockIdx.x;
    if (o.status[r] != 0) return;  // every weight vanished: nothing to learn from
    extern __shared__ __align__(16) unsigned char smem[];
    MlpAct* A = reinterpret_cast<MlpAct*>(smem + sizeof(MlpW));
    __shared__ double red[16 * (2 * DMAX + 1)];
    __shared__ double frs[DMAX + DMAX * DMAX];
    mlp_train_prologue<D>(m, p, o, r, A, red, frs);
}

// the minibatch gradient (the nsub_b sub-batch gradients summed in order), its global
// norm clipped to MLP_CLIP, and one Adam step on the master weights of run r, by one
// 256-thread workgroup (red: block-reduction LDS)
template <int D>
__device__ __forceinline__ void mlp_adam_step(const MlpArrays& m, const MlpParams& p, int r, int nsub_b, double* red)
{
    const int tid = (int)threadIdx.x;
    const int NP = mlp_nparams(D);
    const float* gp = m.gpart + (size_t)r * p.nsub * NP;
    float* grad = m.grad + (size_t)r * NP;
    float* prm = m.params + (size_t)r * NP;
    float* am = m.adam_m + (size_t)r * NP;
    float* av = m.adam_v + (size_t)r * NP;
    // parameters i = tid + 256 e in chunks of CH, every load of a chunk issued first
    constexpr int PER = (mlp_np_const(D) + 255) / 256, CH = 8;
    double nn[1] = {0.0};
#pragma nounroll
    for (int e0 = 0; e0 < PER; e0 += CH) {
        float g[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int i = tid + 256 * (e0 + e);
            g[e] = (e0 + e < PER && i < NP) ? gp[i] : 0.f;
        }
        for (int b = 1; b < nsub_b; ++b) {
            float h[CH];
#pragma unroll
            for (int e = 0; e < CH; ++e) {
                const int i = tid + 256 * (e0 + e);
                h[e] = (e0 + e < PER && i < NP) ? gp[(size_t)b * NP + i] : 0.f;
            }
#pragma unroll
            for (int e = 0; e < CH; ++e) g[e] += h[e];
        }
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int i = tid + 256 * (e0 + e);
            if (e0 + e < PER && i < NP) {
                grad[i] = g[e];
                nn[0] += (double)g[e] * (double)g[e];
            }
        }
    }
    mlp_block_sum<1>(nn, red);
    const double nrm = sqrt(nn[0]);
    const double clip = nrm > MLP_CLIP ? MLP_CLIP / nrm : 1.0;
    const int t_adam = m.adam_t[r] + 1;
    const float c1 = 1.f - powf(0.9f, (float)t_adam), c2 = 1.f - powf(0.999f, (float)t_adam);
#pragma nounroll
    for (int e0 = 0; e0 < PER; e0 += CH) {
        float g[CH], mo[CH], vo[CH], po[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int i = tid + 256 * (e0 + e);
            if (e0 + e < PER && i < NP) {
                g[e] = grad[i];
                mo[e] = am[i];
                vo[e] = av[i];
                po[e] = prm[i];
            }
        }
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int i = tid + 256 * (e0 + e);
            if (e0 + e < PER && i < NP) {
                const float gi = (float)((double)g[e] * clip);
                const float mi = 0.9f * mo[e] + 0.1f * gi;
                const float vi = 0.999f * vo[e] + 0.001f * gi * gi;
                am[i] = mi;
                av[i] = vi;
                prm[i] = po[e] - p.lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
            }
        }
    }
    __syncthreads();  // every thread has read the step count
    if (tid == 0) m.adam_t[r] = t_adam;
}

// gradient of sub-batch blockIdx.x (rows b0 + 64 s .. of the minibatch of nb rows at b0)
// of epoch ep, run blockIdx.y, into m.gpart[r][s]; the last of the minibatch's nsub_b
// workgroups to finish then takes the Adam step (a count per run, no waiting: each
// workgroup releases its gradient device-wide before counting itself, the last one
// acquires before reading them all, and resets the count for the next minibatch)
template <int D>
__global__ void __launch_bounds__(256) k_mlp_sub(MlpArrays m, MlpParams p, OuterArrays o, const uint64_t* seeds,
                                                 int ep, int b0, int nb, int nsub_b)
{
    const int s = (int)blockIdx.x, r = (int)blockIdx.y;
    const int s0 = s * MLP_SUB;
    if (o.status[r] != 0 || s0 >= nb) return;
    const int tid = (int)threadIdx.x;
    const int N = p.N, NP = mlp_nparams(D);
    const int k = *o.k_dev;
    extern __shared__ __align__(16) unsigned char smem[];
    MlpW* W = reinterpret_cast<MlpW*>(smem);
    MlpAct* A = reinterpret_cast<MlpAct*>(smem + sizeof(MlpW));
    mlp_load_weights(D, m.params + (size_t)r * NP, W);
    const float* rows = m.rows + (size_t)r * N * MLP_ROW;
    const double* wfull = m.wfull + (size_t)r * N;
    if (tid < MLP_SUB) {
        uint64_t ta, tb, ia, ib;
        mlp_perm_dev(seeds[r], (uint32_t)k, (uint32_t)ep, 0u, N, ta, tb);
        mlp_perm_dev(seeds[r], (uint32_t)k, (uint32_t)ep, 1u, N, ia, ib);
        float u[MLP_ROW], t[MLP_ROW], wr = 0.f;
#pragma unroll
        for (int d = 0; d < MLP_ROW; ++d) u[d] = t[d] = 0.f;
        if (s0 + tid < nb) {
            const int rr = b0 + s0 + tid;
            const int jt = (int)((ta * (uint64_t)rr + tb) % (uint64_t)N);
            const int ii = (int)((ia * (uint64_t)rr + ib) % (uint64_t)N);
#pragma unroll
            for (int d = 0; d < MLP_ROW; ++d) {
                u[d] = rows[(size_t)ii * MLP_ROW + d];
                t[d] = rows[(size_t)jt * MLP_ROW + d];
            }
            wr = (float)(wfull[jt] / (double)nb);
        }
#pragma unroll
        for (int d = 0; d < 16; ++d) {
            const float ud = d < MLP_ROW ? u[d] : 0.f;
            A->U[tid * LD16 + d] = ud;
            A->TU[d * LDT + tid] = f2bf(ud);
        }
#pragma unroll
        for (int d = 0; d < 8; ++d) A->UT[tid * 8 + d] = t[d];
        A->wr[tid] = wr;
    }
    __syncthreads();
    f32x4 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bb3 = 0.f, bb2 = 0.f, bb1 = 0.f;
    mlp_fwd16<true>(W, A, wave_id() * 16);
    if (lane_id() < 16) mlp_row_nll<D>(A, wave_id() * 16 + lane_id(), A->wr[wave_id() * 16 + lane_id()], true);
    wave_sync();
    mlp_copy_ograd(A, wave_id() * 16);
    mlp_bwd16(W, A, wave_id() * 16);
    mlp_bias16(A, wave_id() * 16, bb3, bb2, bb1);
    __syncthreads();
    mlp_wgrad(A, acc);
    __syncthreads();  // the bias sums below reuse the activations' LDS
    float* gp = m.gpart + ((size_t)r * p.nsub + s) * NP;
    mlp_scatter_wgrad<D>(acc, gp);
    mlp_bias_write<D>(A->H1, bb3, bb2, bb1, gp);
    __shared__ int last;
    __shared__ double red[16 * (2 * DMAX + 1)];
    __threadfence();
    __syncthreads();
    if (tid == 0) last = atomicAdd(m.done + r, 1) == nsub_b - 1 ? 1 : 0;
    __syncthreads();
    if (!uniform_bool(last != 0)) return;
    __threadfence();
    mlp_adam_step<D>(m, p, r, nsub_b, red);
    if (tid == 0) m.done[r] = 0;
}

// held-out sums of sub-batch blockIdx.x of run blockIdx.y, into the run's scratch as
// doubles hp[s][2] (at most 512 sub-batches: far inside the run's share of gpart)
template <int D>
__global__ void __launch_bounds__(256) k_mlp_heldout(MlpArrays m, MlpParams p, OuterArrays o, const uint64_t* seeds)
{
    const int s = (int)blockIdx.x, r = (int)blockIdx.y;
    if (o.status[r] != 0) return;
    const int tid = (int)threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    MlpW* W = reinterpret_cast<MlpW*>(smem);
    MlpAct* A = reinterpret_cast<MlpAct*>(smem + sizeof(MlpW));
    __shared__ double red[16 * (2 * DMAX + 1)];
    __shared__ double frs[DMAX + DMAX * DMAX];
    const double* fr = m.frame + (size_t)r * (D + D * D);
    for (int d = tid; d < D + D * D; d += 256) frs[d] = fr[d];
    mlp_load_weights(D, m.params + (size_t)r * mlp_nparams(D), W);
    __syncthreads();
    double sums[2] = {0.0, 0.0};
    mlp_heldout_rows<D>(m, p, o, r, *o.k_dev, seeds[r], W, A, frs, s * MLP_SUB, (s + 1) * MLP_SUB, sums);
    mlp_block_sum<2>(sums, red);
    if (tid == 0) {
        double* hp = reinterpret_cast<double*>(m.gpart + (size_t)r * p.nsub * mlp_nparams(D)) + 2 * (size_t)s;
        hp[0] = sums[0];
        hp[1] = sums[1];
    }
}

// the sub-batches' held-out sums added in order, and the decision (run blockIdx.x)
template <int D>
__global__ void __launch_bounds__(64) k_mlp_heldout_sum(MlpArrays m, MlpParams p, OuterArrays o, int nblk)
{
    const int r = (int)blockIdx.x;
    if (o.status[r] != 0 || threadIdx.x != 0) return;
    const double* hp = reinterpret_cast<const double*>(m.gpart + (size_t)r * p.nsub * mlp_nparams(D));
    double sm = 0.0, sr = 0.0;
    for (int b = 0; b < nblk; ++b) {
        sm += hp[2 * b];
        sr += hp[2 * b + 1];
    }
    mlp_heldout_decide(m, p, o, r, *o.k_dev, sm, sr);
}

template <int D>
__global__ void __launch_bounds__(256) k_mlp_rows_forward(int n, const float* params, const double* frame,
                                                          const double* phi, float* out)
{
    constexpr int P = D + D * (D + 1) / 2;
    extern __shared__ __align__(16) unsigned char smem[];
    MlpW* W = reinterpret_cast<MlpW*>(smem);
    MlpAct* A = reinterpret_cast<MlpAct*>(smem + sizeof(MlpW));
    mlp_load_weights(D, params, W);
    const int row0 = (int)blockIdx.x * MLP_SUB, tid = (int)threadIdx.x;
    if (tid < MLP_SUB) {
        const int i = row0 + tid;
        float u[16];
#pragma unroll
        for (int d = 0; d < 16; ++d) u[d] = 0.f;
        if (i < n) mlp_whiten<D>(frame, phi + (size_t)i * D, u);
#pragma unroll
        for (int d = 0; d < 16; ++d) A->U[tid * LD16 + d] = u[d];
    }
    __syncthreads();
    mlp_fwd16<false>(W, A, wave_id() * 16);
    __syncthreads();
    for (int e = tid; e < MLP_SUB * P; e += (int)blockDim.x) {
        const int rr = e / P, pp = e - rr * P, i = row0 + rr;
        if (i < n) out[(size_t)i * P + pp] = A->O[rr * LD48 + pp];
    }
}

template <int D>
__global__ void __launch_bounds__(256) k_mlp_rows_grad(int n, const float* params, const double* frame,
                                                       const double* phi_in, const double* phi_t, const double* wrow,
                                                       float* grad, double* loss)
{
    extern __shared__ __align__(16) unsigned char smem[];
    MlpW* W = reinterpret_cast<MlpW*>(smem);
    MlpAct* A = reinterpret_cast<MlpAct*>(smem + sizeof(MlpW));
    __shared__ double red[16 * 2];
    const int tid = (int)threadIdx.x;
    mlp_load_weights(D, params, W);
    f32x4 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bb3 = 0.f, bb2 = 0.f, bb1 = 0.f;
    double ls[1] = {0.0};
    __syncthreads();
    for (int s0 = 0; s0 < n; s0 += MLP_SUB) {
        if (tid < MLP_SUB) {
            const int i = s0 + tid;
            const bool valid = i < n;
            float ui[16], ut[8];
#pragma unroll
            for (int d = 0; d < 16; ++d) ui[d] = 0.f;
#pragma unroll
            for (int d = 0; d < 8; ++d) ut[d] = 0.f;
            if (valid) {
                mlp_whiten<D>(frame, phi_in + (size_t)i * D, ui);
                mlp_whiten<D>(frame, phi_t + (size_t)i * D, ut);
            }
#pragma unroll
            for (int d = 0; d < 16; ++d) {
                A->U[tid * LD16 + d] = ui[d];
                A->TU[d * LDT + tid] = f2bf(ui[d]);
            }
#pragma unroll
            for (int d = 0; d < 8; ++d) A->UT[tid * 8 + d] = ut[d];
            A->wr[tid] = valid ? (float)wrow[i] : 0.f;
        }
        __syncthreads();
        mlp_fwd16<true>(W, A, wave_id() * 16);
        if (lane_id() < 16) {
            const int rr = wave_id() * 16 + lane_id();
            const float wv = A->wr[rr];
            const float nll = mlp_row_nll<D>(A, rr, wv, true);
            if (wv != 0.f) ls[0] += (double)wv * (double)nll;
        }
        wave_sync();
        mlp_copy_ograd(A, wave_id() * 16);
        mlp_bwd16(W, A, wave_id() * 16);
        mlp_bias16(A, wave_id() * 16, bb3, bb2, bb1);
        __syncthreads();
        mlp_wgrad(A, acc);
        __syncthreads();
    }
    mlp_scatter_wgrad<D>(acc, grad);
    mlp_bias_write<D>(A->H1, bb3, bb2, bb1, grad);
    mlp_block_sum<1>(ls, red);
    if (tid == 0) *loss = ls[0];
}

// ------------------------------------------------------------------ host side
template <typename Kern> static hipError_t raise_lds(Kern f, size_t bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

#define MLP_DISPATCH(D, CALL)                                                                                   \
    switch (D) {                                                                                                \
    case 1: CALL(1); break;                                                                                     \
    case 2: CALL(2); break;                                                                                     \
    case 3: CALL(3); break;                                                                                     \
    case 4: CALL(4); break;                                                                                     \
    case 5: CALL(5); break;                                                                                     \
    case 6: CALL(6); break;                                                                                     \
    case 7: CALL(7); break;                                                                                     \
    case 8: CALL(8); break;                                                                                     \
    default: return hipErrorInvalidValue;                                                                       \
    }

hipError_t launch_mlp_forward(const MlpArrays& m, const MlpParams& p, const OuterArrays& o, hipStream_t s)
{
    const dim3 grid((unsigned)((p.N + MLP_SUB - 1) / MLP_SUB), (unsigned)p.R);
    hipError_t e = hipSuccess;
#define CALL_FWD(DD) hipLaunchKernelGGL(k_mlp_forward<DD>, grid, dim3(256), MLP_LDS_FWD, s, m, p, o);
    MLP_DISPATCH(p.D, CALL_FWD)
#undef CALL_FWD
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_mlp_train(const MlpArrays& m, const MlpParams& p, const OuterArrays& o, const uint64_t* seeds,
                            hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (!p.split) {
#define CALL_TRAIN(DD)                                                                                          \
    hipLaunchKernelGGL(k_mlp_train<DD>, dim3((unsigned)p.R), dim3(256), MLP_LDS_TRAIN, s, m, p, o, seeds);
        MLP_DISPATCH(p.D, CALL_TRAIN)
#undef CALL_TRAIN
        return e != hipSuccess ? e : hipGetLastError();
    }
    const int N = p.N, B = (p.batch < 1 || p.batch > N) ? N : p.batch;
    const dim3 runs((unsigned)p.R);
#define CALL_PREP(DD) hipLaunchKernelGGL(k_mlp_prep<DD>, runs, dim3(256), MLP_LDS_TRAIN, s, m, p, o);
    MLP_DISPATCH(p.D, CALL_PREP)
#undef CALL_PREP
    e = hipGetLastError();
    for (int ep = 0; ep < p.epochs && e == hipSuccess; ++ep) {
        for (int b0 = 0; b0 < N && e == hipSuccess; b0 += B) {
            const int nb = (N - b0) < B ? (N - b0) : B;
            const int nsub_b = (nb + MLP_SUB - 1) / MLP_SUB;
            const dim3 grid((unsigned)nsub_b, (unsigned)p.R);
#define CALL_STEP(DD)                                                                                           \
    hipLaunchKernelGGL(k_mlp_sub<DD>, grid, dim3(256), MLP_LDS_TRAIN, s, m, p, o, seeds, ep, b0, nb, nsub_b);
            MLP_DISPATCH(p.D, CALL_STEP)
#undef CALL_STEP
            e = hipGetLastError();
        }
    }
    const int nblk = (N + MLP_SUB - 1) / MLP_SUB;
#define CALL_HELD(DD)                                                                                           \
    hipLaunchKernelGGL(k_mlp_heldout<DD>, dim3((unsigned)nblk, (unsigned)p.R), dim3(256), MLP_LDS_TRAIN, s, m, p, o, \
                       seeds);                                                                                  \
    hipLaunchKernelGGL(k_mlp_heldout_sum<DD>, runs, dim3(64), 0, s, m, p, o, nblk);
    if (e == hipSuccess) {
        MLP_DISPATCH(p.D, CALL_HELD)
    }
#undef CALL_HELD
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_mlp_rows_forward(int D, int n, const float* params, const double* frame, const double* phi,
                                   float* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + MLP_SUB - 1) / MLP_SUB));
    hipError_t e = hipSuccess;
#define CALL_RF(DD) hipLaunchKernelGGL(k_mlp_rows_forward<DD>, grid, dim3(256), MLP_LDS_FWD, s, n, params, frame, phi, out);
    MLP_DISPATCH(D, CALL_RF)
#undef CALL_RF
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_mlp_rows_grad(int D, int n, const float* params, const double* frame, const double* phi_in,
                                const double* phi_t, const double* wrow, float* grad, double* loss, hipStream_t s)
{
    hipError_t e = hipSuccess;
#define CALL_RG(DD)                                                                                             \
    hipLaunchKernelGGL(k_mlp_rows_grad<DD>, dim3(1), dim3(256), MLP_LDS_TRAIN, s, n, params, frame, phi_in, phi_t, \
                       wrow, grad, loss);
    MLP_DISPATCH(D, CALL_RG)
#undef CALL_RG
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t mlp_prepare(int D)
{
    hipError_t e = hipSuccess;
#define CALL_PREP(DD)                                                                                           \
    e = raise_lds(k_mlp_forward<DD>, MLP_LDS_FWD);                                                              \
    if (e == hipSuccess) e = raise_lds(k_mlp_train<DD>, MLP_LDS_TRAIN);                                         \
    if (e == hipSuccess) e = raise_lds(k_mlp_prep<DD>, MLP_LDS_TRAIN);                                          \
    if (e == hipSuccess) e = raise_lds(k_mlp_sub<DD>, MLP_LDS_TRAIN);                                           \
    if (e == hipSuccess) e = raise_lds(k_mlp_heldout<DD>, MLP_LDS_TRAIN);                                       \
    if (e == hipSuccess) e = raise_lds(k_mlp_rows_forward<DD>, MLP_LDS_FWD);                                    \
    if (e == hipSuccess) e = raise_lds(k_mlp_rows_grad<DD>, MLP_LDS_TRAIN);
    MLP_DISPATCH(D, CALL_PREP)
#undef CALL_PREP
    return e;
}

void mlp_init_host(int D, uint64_t seed, float* w)
{
    const int H = MLP_H, P = mlp_nout(D), n = mlp_nparams(D);
    for (int i = 0; i < n; ++i) {
        const W4 x = philox10((uint32_t)i, 0u, 0u, S_MLP_INIT << 24, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double u = u53(x.x, x.y);
        double bound = 0.0;
        if (i < H * D) bound = 1.0 / sqrt((double)D);
        else if (i >= H * D + H && i < H * D + H + H * H) bound = 1.0 / sqrt((double)H);
        else if (i >= H * D + 2 * H + H * H && i < H * D + 2 * H + H * H + P * H) bound = 0.01 / sqrt((double)H);
        w[i] = (float)((2.0 * u - 1.0) * bound);
    }
    float* b3 = w + (H * D + 2 * H + H * H + P * H);
    const double diag0 = log(expm1(1.0 - (double)MLP_EPS));
    for (int i = 0; i < D; ++i) b3[D + i * (i + 1) / 2 + i] = (float)diag0;
}

}  // namespace smc2
