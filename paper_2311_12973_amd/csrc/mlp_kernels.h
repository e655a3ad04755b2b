// mlp_kernels.h — the learned Gaussian proposal on the matrix cores (gfx950).
//
// A D -> 64 -> 64 -> P tanh network (P = D + D(D+1)/2: mean and packed lower
// Cholesky factor) on sampler coordinates whitened by the population's weighted
// mean and covariance. Matrix products run as v_mfma_f32_16x16x16_bf16: BF16 operands
// (FP32 values rounded to nearest even), FP32 accumulation; biases, activations,
// the loss and the Adam update stay FP32 (master weights FP32).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "outer_kernels.h"

namespace smc2 {

constexpr int MLP_H = 64;
constexpr int MLP_PPAD = 48;  // outputs padded to three 16-wide tiles (P <= 44)
constexpr int MLP_SUB = 64;   // rows per sub-batch: four waves of 16
constexpr int MLP_ROW = 8;    // floats per whitened population row (D <= 8)

inline __host__ __device__ int mlp_nout(int D) { return D + D * (D + 1) / 2; }
constexpr int mlp_np_const(int D)
{
    return MLP_H * D + MLP_H + MLP_H * MLP_H + MLP_H + (D + D * (D + 1) / 2) * MLP_H + D + D * (D + 1) / 2;
}
inline __host__ __device__ int mlp_nparams(int D)
{
    const int P = mlp_nout(D);
    return MLP_H * D + MLP_H + MLP_H * MLP_H + MLP_H + P * MLP_H + P;
}

// Per-run state of the learned proposal.
struct MlpArrays {
    float* params;    // [R][NP] FP32 master weights: W1[H][D] b1[H] W2[H][H] b2[H] W3[P][H] b3[P]
    float* adam_m;    // [R][NP]
    float* adam_v;    // [R][NP]
    float* grad;      // [R][NP] minibatch gradient (scratch)
    int32_t* adam_t;  // [R] Adam steps taken
    double* frame;    // [R][D + D*D] input frame of the current network: mean c, Cholesky F
    int32_t* use;     // [R] 1: the next iteration proposes with the network
    float* out;       // [R][N][P] outputs at the current population
    double* score;    // [R][2] held-out mean weighted NLL (network, random walk)
    float* rows;      // [R][N][MLP_ROW] the population whitened in the current frame (training scratch)
    double* wfull;    // [R][N] N w_i, the normalised weights times N (training scratch)
    float* gpart;     // [R][nsub][NP] gradients of the sub-batches of a minibatch (split training)
    int32_t* done;    // [R] sub-batch workgroups of the current minibatch that have written their
                      //     gradient (split training; the last one takes the Adam step and resets it)
};

struct MlpParams {
    int32_t D, N, R, K;
    int32_t epochs, batch;
    float lr;
    int32_t rec_len;
    int32_t nsub;       // sub-batches of MLP_SUB rows per minibatch: ceil(min(batch, N) / MLP_SUB)
    int32_t split;      // 1: train with a workgroup per sub-batch (few runs), 0: one workgroup per run
    const double* lrw;  // [D][D] lower Cholesky factor of the random-walk covariance (device)
};

// Sub-batches of MLP_SUB rows in a training minibatch of `batch` rows (0 or > N: N).
inline int mlp_nsub(int batch, int N)
{
    const int B = (batch < 1 || batch > N) ? N : batch;
    return (B + MLP_SUB - 1) / MLP_SUB;
}
// Whether training spreads a minibatch's sub-batches over workgroups: layout mode
// SMC2_MLP_TRAIN_* (0 auto: when the runs alone would leave most of the device idle).
inline bool mlp_split(int mode, int n_runs) { return mode == 2 || (mode == 0 && n_runs <= 32); }

// Network outputs at the current population, for runs that propose with it at this
// iteration (k >= 2 and use = 1); other runs are skipped on the device.
hipError_t launch_mlp_forward(const MlpArrays& m, const MlpParams& p, const OuterArrays& o, hipStream_t s);
// Training after the outer update (one workgroup per run), then the held-out check
// that sets `use` for the next iteration and record column rec_len - 1.
hipError_t launch_mlp_train(const MlpArrays& m, const MlpParams& p, const OuterArrays& o, const uint64_t* seeds,
                            hipStream_t s);

// Kernel-level: outputs of n rows phi[n][D] under (params, frame = c[D], F[D][D]), out[n][P].
hipError_t launch_mlp_rows_forward(int D, int n, const float* params, const double* frame, const double* phi,
                                   float* out, hipStream_t s);
// Kernel-level: summed parameter gradient (and summed weighted NLL) of n rows with
// inputs phi_in, targets phi_t and row weights wrow (the loss is sum_r wrow_r NLL_r).
hipError_t launch_mlp_rows_grad(int D, int n, const float* params, const double* frame, const double* phi_in,
                                const double* phi_t, const double* wrow, float* grad, double* loss, hipStream_t s);

// Raises the dynamic-LDS limit of the kernels for dimension D (host; call before
// launching or capturing them).
hipError_t mlp_prepare(int D);

// Initial parameters (host), from the learned proposal's Philox stream.
void mlp_init_host(int D, uint64_t seed, float* w);

}  // namespace smc2
