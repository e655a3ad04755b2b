// pf_kernel.h — launch interface of the particle-filter batch kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace smc2 {

enum : int { MODEL_SIR = 0, MODEL_SEIR = 1, MODEL_AGE = 2, MODEL_LG = 3 };

// One run of the batch: its observations start at word y_off of the concatenated
// 32-bit words (T x n_obs counts; for the linear-Gaussian model T FP64 values, low
// word first).
struct RunDev {
    int32_t T;
    int32_t nx;
    int32_t y_off;
    int32_t pad;
    uint32_t k0, k1; // Philox key (run seed)
};

struct PFArgs {
    const double* theta;    // [G][D] model parameters of the G filters
    const uint8_t* active;  // [G] 0 = skip (log-likelihood -inf); NULL = all active
    double* ll;             // [G] log-likelihood estimates (out)
    const int32_t* y;       // concatenated observations of all runs
    const RunDev* runs;     // [n_runs]
    const int32_t* items;   // [n_items] global filter indices g, or NULL for g = item
    const int32_t* k_dev;   // iteration counter in device memory, or NULL to use k_const
    double* trace_inc;      // [G][T] per-day likelihood increments, or NULL (diagnostics)
    int32_t* trace_rs;      // [G][T] per-day resampling flags, or NULL
    int32_t* trace_state;   // [G][T][NC][nx] per-day counts before resampling, or NULL
    int32_t* trace_anc;     // [G][T][nx] ancestors chosen after each day (identity without
                            // resampling; unwritten after a filter's death day), or NULL
    unsigned long long* psteps;  // [n_runs] executed particle-steps: each filter adds N_x x
                                 // the days it ran (to its death day), or NULL
    double* score;          // [G][D] score estimates (score launches only)
    int32_t* queue;         // work-list counter (zero at launch) for a persistent grid, or NULL
    uint32_t k_const;
    int32_t n_items;
    int32_t N;              // filters per run: g = run * N + filter
    int32_t D;
    int32_t pf_always;
    int32_t multinomial;    // 1: multinomial resampling, 0: systematic
    float prio_scale;       // 1 / largest T_r * N_x,r of the launch: wave priority from the
                            // filter's remaining work (0: leave the priority alone)
    double n_pop;
    double fx[32];          // model constants
};

// How a workgroup schedules the binomial draws of a day: every lane finishes its own
// draws in turn, or (SIR, SEIR) the wave pools the draws and batches the final
// acceptance tests of the BTRS sampler. Both give identical flows.
enum : int { PF_SCHED_AUTO = 0, PF_SCHED_PER_DRAW = 1, PF_SCHED_POOLED = 2 };
// Internal launch variants that also carry each particle's running score of its
// trajectory and write the filter's score estimate: on the per-draw schedule (SIR, SEIR
// and the linear-Gaussian model) and on the pooled one (SIR, SEIR; the score terms are
// added when the drawn flows are applied, in the per-draw variant's order, so the two
// give the same bits). Not values of smc2_config.schedule.
constexpr int PF_SCHED_SCORE = 3;
constexpr int PF_SCHED_SCORE_POOLED = 4;
// score coordinates kept per particle: SIR 2, SEIR 5 (iota's stays 0, r's is used when
// r is estimated), linear-Gaussian 3; 0 where the score is not supported
int pf_score_dims(int model);
// dynamic LDS budget of one workgroup (the kernel adds a few bytes of static LDS)
constexpr size_t PF_LDS_MAX = 160 * 1024 - 256;

// Dynamic LDS bytes of one filter workgroup.
size_t pf_lds_bytes(int model, int prec, int block, int nx, int T, int sched);
// The kernel variant to run for a requested draw schedule (PF_SCHED_AUTO: pooled where
// supported and it fits in LDS), with score = true its score-carrying form; -1 when
// the pooled schedule was requested but cannot run, or the model has no score.
int pf_pick_schedule(int model, int prec, int block, int nx, int T, int requested, bool score = false);
// Default workgroup size for a filter of this shape (64 .. 1024 threads).
int pf_default_block(int model, int prec, int nx, int T, int requested_sched, bool score = false);
bool pf_supported(int model, int obs);
// Raise the dynamic-LDS limit of the kernel when a launch needs more than 64 KiB.
hipError_t pf_prepare(int prec, int model, int obs, int sched, size_t lds);
hipError_t launch_pf(int prec, int model, int obs, int sched, int block, size_t lds, const PFArgs& a,
                     hipStream_t s, int grid = 0);
// Workgroups of this configuration resident per CU (for sizing a persistent grid).
hipError_t pf_occupancy(int prec, int model, int obs, int sched, int block, size_t lds, int* per_cu);

}  // namespace smc2
