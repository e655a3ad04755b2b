// smc2_api.cpp — host side of the C ABI declared in include/smc2.h.
//
// Owns validation, the carving of the caller's device workspace, the work list of
// particle filters, the per-iteration launch sequence (optionally replayed as one
// captured HIP graph) and the host-side recycling of the per-iteration records
// (Sec. IV-C). Everything per sample and per particle runs in the device kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/smc2.h"
#include "mlp_kernels.h"
#include "obs_words.h"
#include "outer_kernels.h"
#include "pf_kernel.h"
#include "pmcmc_kernels.h"

using namespace smc2;

namespace {

thread_local std::string g_thread_error;

int expected_D(int model, int D)
{
    if (model == SMC2_SIR) return 2;
    if (model == SMC2_SEIR) return (D == 5) ? 5 : 4;
    if (model == SMC2_AGE_SEIR) return 8;
    if (model == SMC2_LINGAUSS) return 3;
    return -1;
}

// Lower Cholesky factor (row-major); false when not positive definite.
bool host_cholesky(int n, const double* A, double* L)
{
    for (int i = 0; i < n * n; ++i) L[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) return false;
        L[j * n + j] = std::sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = v / L[j * n + j];
        }
    }
    return true;
}

// work-list counters in the workspace: one per launch group, plus one for tuning
constexpr int MAX_GROUPS = 64;
// timing events per iteration: start, after the learned proposal's forward pass, filters
// start and end, after the outer update, end
constexpr int EV_PER_STEP = 6;

struct Layout {
    size_t total = 0;
    size_t off_k, off_status, off_seeds, off_runs, off_y, off_prior, off_lrw, off_phi, off_phin, off_thn, off_lp,
        off_ll, off_logw, off_lpn, off_lln, off_lwp, off_scr, off_qc, off_anc, off_active, off_rec, off_items,
        off_queues, off_tune_items, off_mlp_params, off_mlp_m, off_mlp_v, off_mlp_grad, off_mlp_t, off_mlp_frame,
        off_mlp_use, off_mlp_done, off_mlp_out, off_mlp_logq, off_mlp_score, off_mlp_rows, off_mlp_wfull, off_mlp_gpart,
        off_psteps, off_lkfit, off_psteps_at, off_score, off_score_new, off_pop_chol;
    size_t take(size_t bytes)
    {
        const size_t o = total;
        total += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

Layout make_layout(const smc2_config* c, int R, const smc2_run* runs)
{
    Layout L;
    const size_t N = (size_t)c->N, D = (size_t)c->D, RN = (size_t)R * N;
    size_t ytot = 0;
    for (int r = 0; r < R; ++r) ytot += (size_t)runs[r].T * obs_words(c->model);
    L.off_k = L.take(sizeof(int32_t));
    L.off_status = L.take(sizeof(int32_t) * R);
    L.off_psteps = L.take(sizeof(unsigned long long) * R);
    L.off_lkfit = L.take(sizeof(double) * R * (2 * D + 4 * D * D));
    L.off_psteps_at = L.take(sizeof(unsigned long long) * R * (size_t)c->K);
    L.off_seeds = L.take(sizeof(uint64_t) * R);
    L.off_runs = L.take(sizeof(RunDev) * R);
    L.off_y = L.take(sizeof(int32_t) * ytot);
    L.off_prior = L.take(sizeof(double) * D * 3);
    L.off_lrw = L.take(sizeof(double) * D * D);
    L.off_phi = L.take(sizeof(double) * RN * D);
    L.off_phin = L.take(sizeof(double) * RN * D);
    L.off_thn = L.take(sizeof(double) * RN * D);
    L.off_lp = L.take(sizeof(double) * RN);
    L.off_ll = L.take(sizeof(double) * RN);
    L.off_logw = L.take(sizeof(double) * RN);
    L.off_lpn = L.take(sizeof(double) * RN);
    L.off_lln = L.take(sizeof(double) * RN);
    L.off_lwp = L.take(sizeof(double) * RN);
    L.off_scr = L.take(sizeof(double) * RN);
    L.off_qc = L.take(sizeof(uint64_t) * RN);
    L.off_anc = L.take(sizeof(int32_t) * RN);
    L.off_active = L.take(RN);
    L.off_rec = L.take(sizeof(double) * R * (size_t)c->K * SMC2_RECORD_LEN(c->D));
    L.off_items = L.take(sizeof(int32_t) * RN);
    L.off_queues = L.take(sizeof(int32_t) * MAX_GROUPS);
    L.off_tune_items = L.take(sizeof(int32_t) * RN);
    const bool mlp = c->proposal == SMC2_PROP_MLP;
    const size_t NP = mlp ? (size_t)mlp_nparams(c->D) : 0, P = mlp ? (size_t)mlp_nout(c->D) : 0;
    const size_t Rm = mlp ? (size_t)R : 0;
    L.off_mlp_params = L.take(sizeof(float) * Rm * NP);
    L.off_mlp_m = L.take(sizeof(float) * Rm * NP);
    L.off_mlp_v = L.take(sizeof(float) * Rm * NP);
    L.off_mlp_grad = L.take(sizeof(float) * Rm * NP);
    L.off_mlp_t = L.take(sizeof(int32_t) * Rm);
    L.off_mlp_frame = L.take(sizeof(double) * Rm * (D + D * D));
    L.off_mlp_use = L.take(sizeof(int32_t) * Rm);
    L.off_mlp_done = L.take(sizeof(int32_t) * Rm);
    L.off_mlp_out = L.take(sizeof(float) * Rm * N * P);
    const bool lgv = c->proposal == SMC2_PROP_LANGEVIN;
    const bool popcov = lgv || c->proposal == SMC2_PROP_RW_POP;
    L.off_mlp_logq = L.take(sizeof(double) * (mlp || popcov ? (size_t)R : 0) * N);
    L.off_score = L.take(sizeof(double) * (lgv ? RN * D : 0));
    L.off_score_new = L.take(sizeof(double) * (lgv ? RN * D : 0));
    L.off_pop_chol = L.take(sizeof(double) * (popcov ? (size_t)R * D * D : 0));
    L.off_mlp_score = L.take(sizeof(double) * Rm * 2);
    L.off_mlp_rows = L.take(sizeof(float) * Rm * N * MLP_ROW);
    L.off_mlp_wfull = L.take(sizeof(double) * Rm * N);
    L.off_mlp_gpart = L.take(sizeof(float) * (mlp_split(c->mlp_train, (int)R) ? Rm * (size_t)mlp_nsub(c->mlp_batch, (int)N) * NP : 0));
    return L;
}

// One launch of the particle-filter kernel over a group of filters sharing a block size.
struct PFGroup {
    int block;
    size_t lds;
    int first_item, n_items;
    int sched;       // kernel variant: PF_SCHED_PER_DRAW, PF_SCHED_POOLED or their score forms
    int persistent;  // 1: resident workgroups pull filters from the work list
    int grid;        // workgroups launched when persistent
    int max_nx, max_T;
    float tuned_ms;   // time of the chosen configuration on the tuning sample (0: not tuned)
    double max_cost;  // largest T_r * N_x,r of the group's runs
    long resident;    // workgroups of this configuration resident at once on the device
    float prio;       // PFArgs::prio_scale of the group's launches
};

// Wave-priority scale of a launch of n filters of this group: only when every filter
// is resident at once (the priorities even out the tail of a single round).
float prio_scale(const PFGroup& gr, long n)
{
    return gr.max_cost > 0.0 && n <= gr.resident ? (float)(1.0 / gr.max_cost) : 0.f;
}

}  // namespace

void smc2_set_thread_error(const std::string& m) { g_thread_error = m; }

struct smc2_ctx {
    smc2_config cfg{};
    std::vector<double> prior, rw_cov, fixed;
    std::vector<smc2_run> runs;
    std::vector<std::vector<int32_t>> ys;
    int R = 0;
    int k_host = 0;
    bool poisoned = false;
    std::string err;
    hipStream_t stream = nullptr;
    unsigned char* ws = nullptr;
    Layout lay;
    OuterArrays oa{};
    OuterParams op{};
    MlpArrays ma{};
    MlpParams mp{};
    PFArgs pa{};
    const uint64_t* d_seeds = nullptr;
    std::vector<PFGroup> groups;
    bool graph_ready = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture the graph
    int n_cu = 0;
    std::vector<int32_t> host_items;  // the work list (filter indices), grouped and cost-sorted
    std::vector<hipEvent_t> ev;  // 4 per iteration: step start, pf start, pf end, step end
    int timed_from = 0;

    int fail(int code, const std::string& m)
    {
        err = m;
        g_thread_error = m;
        return code;
    }
    int device_fail(hipError_t e, const char* where)
    {
        poisoned = true;
        return fail(SMC2_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
    }
};

static int validate(const smc2_config* c, int32_t R, const smc2_run* runs, std::string& m)
{
    if (!c || !runs || R < 1) return m = "null config/runs or n_runs < 1", SMC2_E_ARG;
    if (c->model < SMC2_SIR || c->model > SMC2_LINGAUSS) return m = "unknown model", SMC2_E_ARG;
    if (c->obs < SMC2_OBS_POIS_PREV || c->obs > SMC2_OBS_GAUSS) return m = "unknown observation model", SMC2_E_ARG;
    if (!pf_supported(c->model, c->obs)) return m = "model/observation combination not supported", SMC2_E_UNSUPPORTED;
    if (c->D < 1 || c->D > SMC2_DMAX || expected_D(c->model, c->D) != c->D)
        return m = "D does not match the model", SMC2_E_ARG;
    if (c->N < 2 || c->N > 32768) return m = "N must be in [2, 32768]", SMC2_E_ARG;
    if (c->K < 1 || c->K > 65535) return m = "K must be in [1, 65535]", SMC2_E_ARG;
    if (c->precision != SMC2_PREC_FP32 && c->precision != SMC2_PREC_FP64) return m = "bad precision", SMC2_E_ARG;
    const bool lg = c->model == SMC2_LINGAUSS;
    if (lg && c->precision != SMC2_PREC_FP64)
        return m = "the linear-Gaussian model runs in FP64 only", SMC2_E_UNSUPPORTED;
    if (c->proposal != SMC2_PROP_RW && c->proposal != SMC2_PROP_MLP && c->proposal != SMC2_PROP_LANGEVIN &&
        c->proposal != SMC2_PROP_RW_POP)
        return m = "unknown proposal", SMC2_E_UNSUPPORTED;
    if (!(c->lgv_step >= 0.0 && c->lgv_step <= 1.0)) return m = "lgv_step must be in [0, 1]", SMC2_E_ARG;
    if (c->proposal == SMC2_PROP_LANGEVIN && pf_score_dims(c->model) == 0)
        return m = "the Langevin proposal needs the filter's score (SIR, SEIR, linear-Gaussian)", SMC2_E_UNSUPPORTED;
    if (c->proposal == SMC2_PROP_MLP) {
        if (c->mlp_epochs < 0 || c->mlp_epochs > 1000) return m = "mlp_epochs must be in [0, 1000]", SMC2_E_ARG;
        if (c->mlp_batch < 0) return m = "mlp_batch must be >= 0", SMC2_E_ARG;
        if (!(c->mlp_lr > 0.0 && c->mlp_lr < 1.0)) return m = "mlp_lr must be in (0, 1)", SMC2_E_ARG;
    }
    if (c->lkernel != SMC2_L_FORWARD && c->lkernel != SMC2_L_GAUSS_OPT) return m = "unknown L-kernel", SMC2_E_ARG;
    if (!lg && !(c->n_pop >= 1.0 && c->n_pop <= 16777216.0 && c->n_pop == std::floor(c->n_pop)))
        return m = "n_pop must be an integer in [1, 2^24]", SMC2_E_ARG;
    if (c->block != 0 && (c->block < 64 || c->block > 1024 || c->block % 64 != 0))
        return m = "block must be 0 or a multiple of 64 up to 1024", SMC2_E_ARG;
    if (c->schedule < 0 || c->schedule > 2) return m = "schedule must be 0, 1 or 2", SMC2_E_ARG;
    if (c->tune < 0 || c->tune > 1) return m = "tune must be 0 or 1", SMC2_E_ARG;
    if (c->persistent < SMC2_LAUNCH_AUTO || c->persistent > SMC2_LAUNCH_PER_FILTER)
        return m = "persistent must be SMC2_LAUNCH_AUTO, _PERSISTENT or _PER_FILTER", SMC2_E_ARG;
    if (c->pf_resampling != SMC2_PF_RS_SYSTEMATIC && c->pf_resampling != SMC2_PF_RS_MULTINOMIAL)
        return m = "pf_resampling must be SMC2_PF_RS_SYSTEMATIC or SMC2_PF_RS_MULTINOMIAL", SMC2_E_ARG;
    if (c->mlp_train < SMC2_MLP_TRAIN_AUTO || c->mlp_train > SMC2_MLP_TRAIN_SPLIT)
        return m = "mlp_train must be SMC2_MLP_TRAIN_AUTO, _PER_RUN or _SPLIT", SMC2_E_ARG;
    if (c->schedule == 2 && c->model != SMC2_SIR && c->model != SMC2_SEIR)
        return m = "the pooled schedule supports SIR and SEIR only", SMC2_E_UNSUPPORTED;
    if (!c->prior || !c->rw_cov) return m = "prior and rw_cov are required", SMC2_E_ARG;
    if (c->n_fixed < 0 || c->n_fixed > SMC2_NFIXED || (c->n_fixed > 0 && !c->fixed))
        return m = "bad fixed constants", SMC2_E_ARG;
    for (int d = 0; d < c->D; ++d) {
        const int fam = (int)c->prior[3 * d];
        if (fam < SMC2_PRIOR_UNIFORM || fam > SMC2_PRIOR_NORMAL || (double)fam != c->prior[3 * d])
            return m = "bad prior family", SMC2_E_ARG;
        if (fam == SMC2_PRIOR_UNIFORM && !(c->prior[3 * d + 2] > c->prior[3 * d + 1]))
            return m = "uniform prior needs a < b", SMC2_E_ARG;
        if (fam != SMC2_PRIOR_UNIFORM && !(c->prior[3 * d + 2] > 0.0))
            return m = "Gaussian prior needs b > 0", SMC2_E_ARG;
    }
    double L[SMC2_DMAX * SMC2_DMAX];
    if (!host_cholesky(c->D, c->rw_cov, L)) return m = "rw_cov is not positive definite", SMC2_E_ARG;
    const int need_fixed = c->model == SMC2_SIR ? 1
                         : c->model == SMC2_SEIR ? (c->D == 4 ? 1 : 0)
                         : c->model == SMC2_LINGAUSS ? 2 : 20;
    if (c->n_fixed < need_fixed) return m = "missing model constants in fixed", SMC2_E_ARG;
    if (c->model == SMC2_SIR && !(c->fixed[0] >= 0 && c->fixed[0] <= c->n_pop))
        return m = "I_0 out of range", SMC2_E_ARG;
    if (c->model == SMC2_SEIR && c->D == 4 && !(c->fixed[0] > 0)) return m = "dispersion r must be > 0", SMC2_E_ARG;
    if (lg && !(std::isfinite(c->fixed[0]) && c->fixed[1] >= 0 && std::isfinite(c->fixed[1])))
        return m = "the initial state needs a finite mean and a finite standard deviation >= 0", SMC2_E_ARG;
    const int nxmax = c->model == SMC2_AGE_SEIR ? 2048 : 4096;
    for (int r = 0; r < R; ++r) {
        if (runs[r].T < 1 || runs[r].T > 1024) return m = "T must be in [1, 1024]", SMC2_E_ARG;
        if (runs[r].n_x < 1 || runs[r].n_x > nxmax) return m = "n_x out of range", SMC2_E_ARG;
        if (const char* why = obs_check(c->model, runs[r])) return m = why, SMC2_E_ARG;
    }
    return SMC2_OK;
}


extern "C" size_t smc2_workspace_bytes(const smc2_config* cfg, int32_t n_runs, const smc2_run* runs)
{
    std::string m;
    if (validate(cfg, n_runs, runs, m) != SMC2_OK) {
        g_thread_error = m;
        return 0;
    }
    return make_layout(cfg, n_runs, runs).total;
}

// Launch shape of a group: the workgroups resident at once; without the autotuner and with
// SMC2_LAUNCH_AUTO, a persistent grid when the group has more filters than fit at once (at
// the age-structured shape, 16384 filters of one workgroup per CU, 1419 against 1501 ms
// per launch with a workgroup per filter; the same within noise for a single round); the
// persistent grid (all resident workgroups, at most one per filter) and the wave-priority
// scale.
static hipError_t set_launch(smc2_ctx* c, PFGroup& gr)
{
    int per_cu = 0;
    const hipError_t e = pf_occupancy(c->cfg.precision, c->cfg.model, c->cfg.obs, gr.sched, gr.block, gr.lds, &per_cu);
    if (e != hipSuccess) return e;
    gr.resident = (long)(per_cu > 0 ? per_cu : 1) * (c->n_cu > 0 ? c->n_cu : 1);
    if (!c->cfg.tune && c->cfg.persistent == SMC2_LAUNCH_AUTO) gr.persistent = gr.n_items > gr.resident ? 1 : 0;
    if (gr.persistent) gr.grid = (int)std::min<long>(gr.resident, gr.n_items);
    gr.prio = prio_scale(gr, gr.n_items);
    return hipSuccess;
}

// Autotuner: for every launch group, time each candidate (workgroup size, draw
// schedule, persistent or one-filter-per-workgroup grid) on a sample of the group's
// filters at the first iteration's parameters (prior draws) and keep the fastest.
// Results do not depend on the choice (every draw is a function of its coordinates),
// only the time does. Leaves the sampler state as smc2_init found it (k = 0).
static hipError_t autotune(smc2_ctx* c)
{
    const smc2_config& cfg = c->cfg;
    hipStream_t s = c->stream;
    unsigned char* w = c->ws;
    const int32_t one = 1;
    hipError_t e = hipMemcpyAsync(w + c->lay.off_k, &one, sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_propose(c->oa, c->op, c->d_seeds, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    int32_t* d_tune = (int32_t*)(w + c->lay.off_tune_items);
    int32_t* d_queue = (int32_t*)(w + c->lay.off_queues) + (MAX_GROUPS - 1);
    const std::vector<int32_t>& host_items = c->host_items;
    for (PFGroup& gr : c->groups) {
        if (e != hipSuccess) break;
        // sample: about two resident waves of workgroups, strided over the cost-sorted list
        int per_cu = 1;
        e = pf_occupancy(cfg.precision, cfg.model, cfg.obs, gr.sched, gr.block, gr.lds, &per_cu);
        if (e != hipSuccess) break;
        const int S = std::min(gr.n_items, std::max(64, 2 * std::max(per_cu, 1) * std::max(c->n_cu, 1)));
        std::vector<int32_t> sample(S);
        for (int i = 0; i < S; ++i) sample[i] = host_items[gr.first_item + (int)((long)i * gr.n_items / S)];
        e = hipMemcpyAsync(d_tune, sample.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, s);
        PFGroup best = gr;
        float best_ms = -1.f;
        const int full = ((gr.max_nx + 63) / 64) * 64;
        for (int b = 64; b <= 1024 && e == hipSuccess; b *= 2) {
            if (b > std::max(64, full)) break;
            for (int sc = PF_SCHED_PER_DRAW; sc <= PF_SCHED_SCORE_POOLED && e == hipSuccess; ++sc) {
                // the Langevin proposal's launches carry the scores: only those variants
                const bool sc_score = sc == PF_SCHED_SCORE || sc == PF_SCHED_SCORE_POOLED;
                const bool sc_pooled = sc == PF_SCHED_POOLED || sc == PF_SCHED_SCORE_POOLED;
                if ((cfg.proposal == SMC2_PROP_LANGEVIN) != sc_score) continue;
                if (cfg.schedule != SMC2_SCHED_AUTO &&
                    (sc_pooled ? SMC2_SCHED_POOLED : SMC2_SCHED_PER_DRAW) != cfg.schedule)
                    continue;
                if (sc_pooled && cfg.model != SMC2_SIR && cfg.model != SMC2_SEIR) continue;
                const size_t lds = pf_lds_bytes(cfg.model, cfg.precision, b, gr.max_nx, gr.max_T, sc);
                if (lds > PF_LDS_MAX) continue;
                e = pf_prepare(cfg.precision, cfg.model, cfg.obs, sc, lds);
                for (int pers = 0; pers <= 1 && e == hipSuccess; ++pers) {
                    PFGroup cand = gr;
                    cand.block = b;
                    cand.sched = sc;
                    cand.lds = lds;
                    cand.persistent = pers;
                    e = set_launch(c, cand);
                    if (e != hipSuccess) break;
                    PFArgs a = c->pa;
                    a.items = d_tune;
                    a.n_items = S;
                    a.k_dev = nullptr;
                    a.k_const = 1;
                    a.queue = pers ? d_queue : nullptr;
                    a.prio_scale = prio_scale(cand, S);
                    int grid = pers ? std::min(cand.grid, S) : 0;
                    float ms = -1.f;
                    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {  // rep 0 warms up
                        if (pers) e = hipMemsetAsync(d_queue, 0, sizeof(int32_t), s);
                        if (e == hipSuccess) e = hipEventRecord(t0, s);
                        if (e == hipSuccess) e = launch_pf(cfg.precision, cfg.model, cfg.obs, sc, b, lds, a, s, grid);
                        if (e == hipSuccess) e = hipEventRecord(t1, s);
                        if (e == hipSuccess) e = hipEventSynchronize(t1);
                        float t = 0.f;
                        if (e == hipSuccess) e = hipEventElapsedTime(&t, t0, t1);
                        if (rep > 0 && (ms < 0.f || t < ms)) ms = t;
                    }
                    if (e == hipSuccess && (best_ms < 0.f || ms < best_ms)) {
                        best_ms = ms;
                        best = cand;
                    }
                }
            }
        }
        if (e == hipSuccess && best_ms >= 0.f) {
            // the chosen size must hold every run of the group
            best.lds = 0;
            gr = best;
            gr.tuned_ms = best_ms;
        }
    }
    // recompute the LDS of each group for all its runs under the chosen configuration
    for (PFGroup& gr : c->groups) {
        if (e != hipSuccess) break;
        if (gr.lds == 0) {
            for (int i = 0; i < gr.n_items; ++i) {
                const int r = host_items[gr.first_item + i] / cfg.N;
                gr.lds = std::max(gr.lds, pf_lds_bytes(cfg.model, cfg.precision, gr.block, c->runs[r].n_x,
                                                       c->runs[r].T, gr.sched));
            }
            if (gr.lds > PF_LDS_MAX) return hipErrorInvalidValue;
            e = pf_prepare(cfg.precision, cfg.model, cfg.obs, gr.sched, gr.lds);
        }
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (e == hipSuccess) e = hipMemsetAsync(w + c->lay.off_k, 0, sizeof(int32_t), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

extern "C" int smc2_init(const smc2_config* cfg, int32_t n_runs, const smc2_run* runs, void* d_workspace,
                         size_t ws_bytes, void* hip_stream, smc2_ctx** out)
{
    if (!out) return g_thread_error = "out is NULL", SMC2_E_ARG;
    *out = nullptr;
    std::string m;
    const int v = validate(cfg, n_runs, runs, m);
    if (v != SMC2_OK) return g_thread_error = m, v;
    const Layout lay = make_layout(cfg, n_runs, runs);
    if (!d_workspace || ws_bytes < lay.total || ((uintptr_t)d_workspace & 255u) != 0)
        return g_thread_error = "workspace missing, too small or not 256-byte aligned", SMC2_E_ARG;

    smc2_ctx* c = new smc2_ctx();
    c->cfg = *cfg;
    c->R = n_runs;
    c->prior.assign(cfg->prior, cfg->prior + 3 * cfg->D);
    c->rw_cov.assign(cfg->rw_cov, cfg->rw_cov + cfg->D * cfg->D);
    c->fixed.assign(SMC2_NFIXED, 0.0);
    for (int i = 0; i < cfg->n_fixed; ++i) c->fixed[i] = cfg->fixed[i];
    c->cfg.prior = c->prior.data();
    c->cfg.rw_cov = c->rw_cov.data();
    c->cfg.fixed = c->fixed.data();
    c->stream = (hipStream_t)hip_stream;
    c->ws = (unsigned char*)d_workspace;
    c->lay = lay;
    c->runs.assign(runs, runs + n_runs);
    std::vector<int32_t> yall;
    std::vector<RunDev> rd(n_runs);
    std::vector<uint64_t> seeds(n_runs);
    for (int r = 0; r < n_runs; ++r) {
        c->ys.emplace_back();
        obs_pack(cfg->model, runs[r], c->ys.back());
        c->runs[r].y = c->ys.back().data();  // the staged words (also for the linear-Gaussian model)
        c->runs[r].y_real = nullptr;
        rd[r].T = runs[r].T;
        rd[r].nx = runs[r].n_x;
        rd[r].y_off = (int32_t)yall.size();
        rd[r].pad = 0;
        rd[r].k0 = (uint32_t)runs[r].seed;
        rd[r].k1 = (uint32_t)(runs[r].seed >> 32);
        seeds[r] = runs[r].seed;
        yall.insert(yall.end(), c->ys.back().begin(), c->ys.back().end());
    }
    std::vector<double> lrw(cfg->D * cfg->D);
    host_cholesky(cfg->D, cfg->rw_cov, lrw.data());

    // work list: filters grouped by workgroup size, longest filters first in each group
    const size_t N = (size_t)cfg->N;
    std::vector<int32_t> items;
    std::vector<int> blk(n_runs);
    // the Langevin proposal needs the filters' scores: their launches carry them
    const bool lgv = cfg->proposal == SMC2_PROP_LANGEVIN;
    const int want = cfg->schedule;
    const int pooled_variant = lgv ? PF_SCHED_SCORE_POOLED : PF_SCHED_POOLED;
    const int per_draw_variant = lgv ? PF_SCHED_SCORE : PF_SCHED_PER_DRAW;
    for (int r = 0; r < n_runs; ++r)
        blk[r] = cfg->block ? cfg->block
                            : pf_default_block(cfg->model, cfg->precision, runs[r].n_x, runs[r].T, want, lgv);
    std::vector<int> run_order(n_runs);
    for (int r = 0; r < n_runs; ++r) run_order[r] = r;
    std::stable_sort(run_order.begin(), run_order.end(), [&](int a, int b) {
        if (blk[a] != blk[b]) return blk[a] > blk[b];
        return (int64_t)runs[a].T * runs[a].n_x > (int64_t)runs[b].T * runs[b].n_x;
    });
    for (size_t idx = 0; idx < run_order.size();) {
        const int b = blk[run_order[idx]];
        PFGroup gr{b, 0, (int)items.size(), 0, pooled_variant, cfg->persistent == SMC2_LAUNCH_PERSISTENT ? 1 : 0,
                   0, 0, 0, 0.f, 0.0, 0, 0.f};
        const size_t g0 = idx;
        // the pooled schedule when every run of the group fits in LDS with it
        for (size_t x = g0; x < run_order.size() && blk[run_order[x]] == b; ++x) {
            const int r = run_order[x];
            const int sc = pf_pick_schedule(cfg->model, cfg->precision, b, runs[r].n_x, runs[r].T, want, lgv);
            if (sc < 0) {
                delete c;
                return g_thread_error = "the pooled schedule does not fit in LDS for this n_x and T", SMC2_E_ARG;
            }
            if (sc == per_draw_variant) gr.sched = per_draw_variant;
        }
        for (; idx < run_order.size() && blk[run_order[idx]] == b; ++idx) {
            const int r = run_order[idx];
            for (size_t i = 0; i < N; ++i) items.push_back((int32_t)(r * N + i));
            gr.lds = std::max(gr.lds, pf_lds_bytes(cfg->model, cfg->precision, b, runs[r].n_x, runs[r].T, gr.sched));
            gr.max_nx = std::max(gr.max_nx, runs[r].n_x);
            gr.max_T = std::max(gr.max_T, runs[r].T);
            gr.max_cost = std::max(gr.max_cost, (double)runs[r].T * (double)runs[r].n_x);
        }
        gr.n_items = (int)items.size() - gr.first_item;
        c->groups.push_back(gr);
    }
    c->host_items = items;
    if ((int)c->groups.size() > MAX_GROUPS - 1) {
        delete c;
        return g_thread_error = "too many distinct workgroup sizes", SMC2_E_ARG;
    }
    for (const PFGroup& gr : c->groups) {
        if (gr.lds > PF_LDS_MAX) {
            delete c;
            return g_thread_error = "particle filter does not fit in LDS (n_x or T too large)", SMC2_E_ARG;
        }
        const hipError_t e = pf_prepare(cfg->precision, cfg->model, cfg->obs, gr.sched, gr.lds);
        if (e != hipSuccess) {
            const int rc = c->device_fail(e, "pf_prepare");
            g_thread_error = c->err;
            delete c;
            return rc;
        }
    }

    unsigned char* w = c->ws;
    OuterArrays& o = c->oa;
    o.phi = (double*)(w + lay.off_phi);
    o.lp = (double*)(w + lay.off_lp);
    o.ll = (double*)(w + lay.off_ll);
    o.logw = (double*)(w + lay.off_logw);
    o.phi_new = (double*)(w + lay.off_phin);
    o.lp_new = (double*)(w + lay.off_lpn);
    o.ll_new = (double*)(w + lay.off_lln);
    o.theta_new = (double*)(w + lay.off_thn);
    o.logw_pre = (double*)(w + lay.off_lwp);
    o.scratch = (double*)(w + lay.off_scr);
    o.qc = (uint64_t*)(w + lay.off_qc);
    o.anc = (int32_t*)(w + lay.off_anc);
    o.active = (uint8_t*)(w + lay.off_active);
    o.records = (double*)(w + lay.off_rec);
    o.status = (int32_t*)(w + lay.off_status);
    o.lkfit = (double*)(w + lay.off_lkfit);
    o.psteps = (const unsigned long long*)(w + lay.off_psteps);
    o.psteps_at = (unsigned long long*)(w + lay.off_psteps_at);
    o.k_dev = (int32_t*)(w + lay.off_k);
    const bool mlp = cfg->proposal == SMC2_PROP_MLP;
    if (mlp) {
        MlpArrays& ma = c->ma;
        ma.params = (float*)(w + lay.off_mlp_params);
        ma.adam_m = (float*)(w + lay.off_mlp_m);
        ma.adam_v = (float*)(w + lay.off_mlp_v);
        ma.grad = (float*)(w + lay.off_mlp_grad);
        ma.adam_t = (int32_t*)(w + lay.off_mlp_t);
        ma.frame = (double*)(w + lay.off_mlp_frame);
        ma.use = (int32_t*)(w + lay.off_mlp_use);
        ma.out = (float*)(w + lay.off_mlp_out);
        ma.score = (double*)(w + lay.off_mlp_score);
        ma.rows = (float*)(w + lay.off_mlp_rows);
        ma.wfull = (double*)(w + lay.off_mlp_wfull);
        ma.gpart = (float*)(w + lay.off_mlp_gpart);
        ma.done = (int32_t*)(w + lay.off_mlp_done);
        o.mlp_use = ma.use;
        o.mlp_out = ma.out;
        o.mlp_frame = ma.frame;
        o.logq = (double*)(w + lay.off_mlp_logq);
    }
    const bool popcov = lgv || cfg->proposal == SMC2_PROP_RW_POP;
    if (popcov) {
        o.logq = (double*)(w + lay.off_mlp_logq);
        o.pop_chol = (double*)(w + lay.off_pop_chol);
    }
    if (lgv) {
        o.score = (double*)(w + lay.off_score);
        o.score_new = (double*)(w + lay.off_score_new);
    }
    OuterParams& p = c->op;
    p.N = cfg->N;
    p.D = cfg->D;
    p.K = cfg->K;
    p.R = n_runs;
    p.lkernel = cfg->lkernel;
    p.rec_len = SMC2_RECORD_LEN(cfg->D);
    p.prior = (const double*)(w + lay.off_prior);
    p.lrw = (const double*)(w + lay.off_lrw);
    p.mlp = mlp ? 1 : 0;
    p.langevin = lgv ? 1 : 0;
    p.popcov = popcov ? 1 : 0;
    p.lgv_step = cfg->lgv_step > 0.0 ? cfg->lgv_step : 0.25;
    {
        MlpParams& q = c->mp;
        q.D = cfg->D;
        q.N = cfg->N;
        q.R = n_runs;
        q.K = cfg->K;
        q.epochs = cfg->mlp_epochs;
        q.batch = cfg->mlp_batch;
        q.lr = (float)cfg->mlp_lr;
        q.rec_len = SMC2_RECORD_LEN(cfg->D);
        q.nsub = mlp_nsub(cfg->mlp_batch, cfg->N);
        q.split = mlp_split(cfg->mlp_train, n_runs) ? 1 : 0;
        q.lrw = p.lrw;
    }
    c->d_seeds = (const uint64_t*)(w + lay.off_seeds);
    PFArgs& a = c->pa;
    a.theta = o.theta_new;
    a.active = o.active;
    a.ll = o.ll_new;
    a.y = (const int32_t*)(w + lay.off_y);
    a.runs = (const RunDev*)(w + lay.off_runs);
    a.items = (const int32_t*)(w + lay.off_items);
    a.k_dev = o.k_dev;
    a.k_const = 0;
    a.N = cfg->N;
    a.D = cfg->D;
    a.pf_always = cfg->pf_always;
    a.multinomial = cfg->pf_resampling;
    a.n_pop = cfg->n_pop;
    a.score = lgv ? o.score_new : nullptr;
    for (int i = 0; i < SMC2_NFIXED; ++i) a.fx[i] = c->fixed[i];

    hipStream_t s = c->stream;
    hipError_t e = hipSuccess;
    auto H2D = [&](size_t off, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    H2D(lay.off_seeds, seeds.data(), sizeof(uint64_t) * n_runs);
    H2D(lay.off_runs, rd.data(), sizeof(RunDev) * n_runs);
    H2D(lay.off_y, yall.data(), sizeof(int32_t) * yall.size());
    H2D(lay.off_prior, c->prior.data(), sizeof(double) * c->prior.size());
    H2D(lay.off_lrw, lrw.data(), sizeof(double) * lrw.size());
    H2D(lay.off_items, items.data(), sizeof(int32_t) * items.size());
    std::vector<float> init_params;
    if (mlp && e == hipSuccess) e = mlp_prepare(cfg->D);
    if (mlp) {
        const size_t NP = (size_t)mlp_nparams(cfg->D);
        init_params.resize(NP * n_runs);
        for (int r = 0; r < n_runs; ++r) mlp_init_host(cfg->D, runs[r].seed, init_params.data() + NP * r);
        H2D(lay.off_mlp_params, init_params.data(), sizeof(float) * init_params.size());
        const size_t zero_from = lay.off_mlp_m, zero_to = lay.off_mlp_out;  // moments, grad, steps, frame, use, count
        if (e == hipSuccess) e = hipMemsetAsync(w + zero_from, 0, zero_to - zero_from, s);
        if (e == hipSuccess) e = hipMemsetAsync(w + lay.off_mlp_score, 0, sizeof(double) * 2 * n_runs, s);
    }
    if (lgv && e == hipSuccess) e = hipMemsetAsync(w + lay.off_score, 0, sizeof(double) * n_runs * N * cfg->D, s);
    if (e == hipSuccess) e = hipMemsetAsync(w + lay.off_k, 0, sizeof(int32_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(w + lay.off_status, 0, sizeof(int32_t) * n_runs, s);
    if (e == hipSuccess) e = hipMemsetAsync(w + lay.off_psteps, 0, sizeof(unsigned long long) * n_runs, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(w + lay.off_psteps_at, 0, sizeof(unsigned long long) * n_runs * cfg->K, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(w + lay.off_lkfit, 0, sizeof(double) * n_runs * (2 * cfg->D + 4 * cfg->D * cfg->D), s);
    if (e == hipSuccess) e = hipMemsetAsync(w + lay.off_logw, 0, sizeof(double) * n_runs * N, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(w + lay.off_rec, 0, sizeof(double) * n_runs * cfg->K * SMC2_RECORD_LEN(cfg->D), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && cfg->tune) e = autotune(c);
    for (PFGroup& gr : c->groups) {
        if (e != hipSuccess) break;
        e = set_launch(c, gr);
    }
    if (e == hipSuccess) {
        c->ev.resize(EV_PER_STEP * (size_t)cfg->K, nullptr);
        for (auto& ev : c->ev)
            if (e == hipSuccess) e = hipEventCreate(&ev);
    }
    if (e != hipSuccess) {
        const int rc = c->device_fail(e, "smc2_init");
        g_thread_error = c->err;
        smc2_destroy(c);
        return rc;
    }
    *out = c;
    return SMC2_OK;
}

// ev (NULL inside a graph capture): events [1] after the learned proposal's forward
// pass, [2] before and [3] after the filter launches, [4] after the outer update.
static hipError_t enqueue_iteration(smc2_ctx* c, hipStream_t s, const hipEvent_t* ev)
{
    int32_t* queues = (int32_t*)(c->ws + c->lay.off_queues);
    hipError_t e = launch_begin_iteration(c->oa, queues, (int)c->groups.size(), s);
    if (e == hipSuccess && c->op.mlp) e = launch_mlp_forward(c->ma, c->mp, c->oa, s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess && c->op.popcov) e = launch_pop_frame(c->oa, c->op, s);
    if (e == hipSuccess) e = launch_propose(c->oa, c->op, c->d_seeds, s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2], s);
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        if (e != hipSuccess) break;
        const PFGroup& gr = c->groups[gi];
        PFArgs a = c->pa;
        a.items = c->pa.items + gr.first_item;
        a.n_items = gr.n_items;
        a.queue = gr.persistent ? queues + gi : nullptr;
        a.prio_scale = gr.prio;
        a.psteps = (unsigned long long*)(c->ws + c->lay.off_psteps);
        e = launch_pf(c->cfg.precision, c->cfg.model, c->cfg.obs, gr.sched, gr.block, gr.lds, a, s, gr.grid);
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[3], s);
    if (e == hipSuccess) e = launch_outer_update(c->oa, c->op, c->d_seeds, s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[4], s);
    if (e == hipSuccess && c->op.mlp) e = launch_mlp_train(c->ma, c->mp, c->oa, c->d_seeds, s);
    return e;
}

extern "C" int smc2_step(smc2_ctx* c)
{
    if (!c) return g_thread_error = "ctx is NULL", SMC2_E_ARG;
    if (c->poisoned) return c->fail(SMC2_E_DEVICE, "context poisoned by an earlier device error");
    if (c->k_host >= c->cfg.K) return c->fail(SMC2_E_STATE, "all K iterations have run");
    const int k = c->k_host + 1;
    hipEvent_t* ev = &c->ev[EV_PER_STEP * (size_t)(k - 1)];
    hipError_t e = hipEventRecord(ev[0], c->stream);
    if (e == hipSuccess) {
        if (c->cfg.use_graph) {
            if (!c->graph_ready) {
                // capture on a private stream (the caller's may be the null stream, which
                // cannot be captured); the graph is then replayed on the caller's stream
                if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
                if (e == hipSuccess) e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    const hipError_t e1 = enqueue_iteration(c, c->cap_stream, nullptr);
                    e = hipStreamEndCapture(c->cap_stream, &c->graph);
                    if (e1 != hipSuccess) e = e1;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0);
                if (e == hipSuccess) c->graph_ready = true;
            }
            // the graph's phases are not timed; [2] and [3] bracket the whole graph
            if (e == hipSuccess) e = hipEventRecord(ev[2], c->stream);
            if (e == hipSuccess) e = hipGraphLaunch(c->graph_exec, c->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[3], c->stream);
        } else {
            e = enqueue_iteration(c, c->stream, ev);
        }
    }
    if (e == hipSuccess) e = hipEventRecord(ev[5], c->stream);
    if (e != hipSuccess) return c->device_fail(e, "smc2_step");
    c->k_host = k;
    return SMC2_OK;
}

static int sync_and_status(smc2_ctx* c, int32_t run)
{
    if (c->poisoned) return c->fail(SMC2_E_DEVICE, "context poisoned by an earlier device error");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->device_fail(e, "synchronize");
    int32_t st = 0;
    e = hipMemcpy(&st, c->oa.status + run, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return c->device_fail(e, "status readback");
    return st == 0 ? SMC2_OK : c->fail(SMC2_E_NUMERIC, "every weight of the run vanished");
}

extern "C" int smc2_records(smc2_ctx* c, int32_t run, double* host_dst, size_t n_doubles, int32_t* k_done)
{
    if (!c) return g_thread_error = "ctx is NULL", SMC2_E_ARG;
    if (run < 0 || run >= c->R || !host_dst) return c->fail(SMC2_E_ARG, "bad run or destination");
    const size_t RL = SMC2_RECORD_LEN(c->cfg.D);
    if (n_doubles < (size_t)c->k_host * RL) return c->fail(SMC2_E_ARG, "destination too small");
    const int st = sync_and_status(c, run);
    if (st == SMC2_E_DEVICE) return st;
    const hipError_t e = hipMemcpy(host_dst, c->oa.records + (size_t)run * c->cfg.K * RL,
                                   sizeof(double) * RL * c->k_host, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return c->device_fail(e, "records readback");
    if (k_done) *k_done = c->k_host;
    return st;
}

extern "C" int smc2_estimate(smc2_ctx* c, int32_t run, int32_t recycled, double* mean, double* cov)
{
    if (!c) return g_thread_error = "ctx is NULL", SMC2_E_ARG;
    if (!mean) return c->fail(SMC2_E_ARG, "mean is NULL");
    if (c->k_host < 1) return c->fail(SMC2_E_STATE, "no iteration has run");
    const int D = c->cfg.D;
    const size_t RL = SMC2_RECORD_LEN(D);
    std::vector<double> rec(RL * c->k_host);
    int32_t kd = 0;
    const int st = smc2_records(c, run, rec.data(), rec.size(), &kd);
    if (st != SMC2_OK) return st;
    // c_k = l_k / sum_j l_j over the completed iterations (Sec. IV-C); mean = sum c_k f_k,
    // covariance = sum c_k (C_k + f_k f_k^T) - mean mean^T.
    const int k0 = recycled ? 0 : kd - 1;
    double lsum = 0.0;
    for (int k = k0; k < kd; ++k) lsum += rec[k * RL + 1];
    std::vector<double> m(D, 0.0), C(D * D, 0.0);
    for (int k = k0; k < kd; ++k) {
        const double ck = rec[k * RL + 1] / lsum;
        const double* fk = &rec[k * RL + 6];
        const double* Ck = &rec[k * RL + 6 + D];
        for (int a = 0; a < D; ++a) m[a] += ck * fk[a];
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) C[a * D + b] += ck * (Ck[a * D + b] + fk[a] * fk[b]);
    }
    for (int a = 0; a < D; ++a) mean[a] = m[a];
    if (cov)
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) cov[a * D + b] = C[a * D + b] - m[a] * m[b];
    return SMC2_OK;
}

extern "C" int smc2_dump(smc2_ctx* c, int32_t what, int32_t run, void* host_dst, size_t bytes)
{
    if (!c) return g_thread_error = "ctx is NULL", SMC2_E_ARG;
    if (run < 0 || run >= c->R || !host_dst) return c->fail(SMC2_E_ARG, "bad run or destination");
    const size_t N = (size_t)c->cfg.N, D = (size_t)c->cfg.D, base = (size_t)run * N;
    const void* src = nullptr;
    size_t need = 0;
    switch (what) {
    case SMC2_DUMP_PHI: src = c->oa.phi + base * D; need = N * D * 8; break;
    case SMC2_DUMP_LP: src = c->oa.lp + base; need = N * 8; break;
    case SMC2_DUMP_LL: src = c->oa.ll + base; need = N * 8; break;
    case SMC2_DUMP_LOGW: src = c->oa.logw + base; need = N * 8; break;
    case SMC2_DUMP_PHI_NEW: src = c->oa.phi_new + base * D; need = N * D * 8; break;
    case SMC2_DUMP_THETA_NEW: src = c->oa.theta_new + base * D; need = N * D * 8; break;
    case SMC2_DUMP_LP_NEW: src = c->oa.lp_new + base; need = N * 8; break;
    case SMC2_DUMP_LL_NEW: src = c->oa.ll_new + base; need = N * 8; break;
    case SMC2_DUMP_LOGW_PRE: src = c->oa.logw_pre + base; need = N * 8; break;
    case SMC2_DUMP_ANC: src = c->oa.anc + base; need = N * 4; break;
    case SMC2_DUMP_PSTEPS: src = c->ws + c->lay.off_psteps + sizeof(unsigned long long) * run; need = 8; break;
    case SMC2_DUMP_LKFIT:
        src = c->oa.lkfit + (size_t)run * (2 * D + 4 * D * D);
        need = (2 * D + 4 * D * D) * 8;
        break;
    case SMC2_DUMP_SCORE:
    case SMC2_DUMP_SCORE_NEW:
        if (!c->op.langevin) return c->fail(SMC2_E_ARG, "the context has no Langevin proposal");
        src = (what == SMC2_DUMP_SCORE ? c->oa.score : c->oa.score_new) + base * D;
        need = N * D * 8;
        break;
    case SMC2_DUMP_MLP_OUT:
    case SMC2_DUMP_LOGQ:
    case SMC2_DUMP_MLP_PARAMS:
    case SMC2_DUMP_MLP_FRAME:
    case SMC2_DUMP_MLP_GRAD:
    case SMC2_DUMP_MLP_STATE: {
        if (what == SMC2_DUMP_LOGQ && c->op.popcov) {
            src = c->oa.logq + base;
            need = N * 8;
            break;
        }
        if (!c->op.mlp) return c->fail(SMC2_E_ARG, "the context has no learned proposal");
        const size_t NP = (size_t)mlp_nparams((int)D), P = (size_t)mlp_nout((int)D);
        if (what == SMC2_DUMP_MLP_OUT) src = c->ma.out + base * P, need = N * P * 4;
        if (what == SMC2_DUMP_LOGQ) src = c->oa.logq + base, need = N * 8;
        if (what == SMC2_DUMP_MLP_PARAMS) src = c->ma.params + (size_t)run * NP, need = NP * 4;
        if (what == SMC2_DUMP_MLP_FRAME) src = c->ma.frame + (size_t)run * (D + D * D), need = (D + D * D) * 8;
        if (what == SMC2_DUMP_MLP_GRAD) src = c->ma.grad + (size_t)run * NP, need = NP * 4;
        if (what == SMC2_DUMP_MLP_STATE) {
            if (bytes < 4 * 8) return c->fail(SMC2_E_ARG, "destination too small");
            if (c->poisoned) return c->fail(SMC2_E_DEVICE, "context poisoned by an earlier device error");
            int32_t ut[2] = {0, 0};
            double sc[2] = {0.0, 0.0};
            hipError_t e = hipStreamSynchronize(c->stream);
            if (e == hipSuccess) e = hipMemcpy(&ut[0], c->ma.use + run, 4, hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(&ut[1], c->ma.adam_t + run, 4, hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(sc, c->ma.score + 2 * (size_t)run, 16, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return c->device_fail(e, "dump");
            double* d = (double*)host_dst;
            d[0] = ut[0];
            d[1] = ut[1];
            d[2] = sc[0];
            d[3] = sc[1];
            return SMC2_OK;
        }
        break;
    }
    default: return c->fail(SMC2_E_ARG, "unknown dump");
    }
    if (bytes < need) return c->fail(SMC2_E_ARG, "destination too small");
    if (c->poisoned) return c->fail(SMC2_E_DEVICE, "context poisoned by an earlier device error");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(host_dst, src, need, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return c->device_fail(e, "dump");
    return SMC2_OK;
}

extern "C" int smc2_timing(smc2_ctx* c, double* ms_pf, double* ms_step, int32_t* n_steps)
{
    if (!c) return g_thread_error = "ctx is NULL", SMC2_E_ARG;
    if (c->poisoned) return c->fail(SMC2_E_DEVICE, "context poisoned by an earlier device error");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->device_fail(e, "synchronize");
    double pf = 0.0, st = 0.0;
    const int n = c->k_host - c->timed_from;
    for (int k = c->timed_from; k < c->k_host; ++k) {
        float a = 0.f, b = 0.f;
        e = hipEventElapsedTime(&a, c->ev[EV_PER_STEP * k + 2], c->ev[EV_PER_STEP * k + 3]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, c->ev[EV_PER_STEP * k + 0], c->ev[EV_PER_STEP * k + 5]);
        if (e != hipSuccess) return c->device_fail(e, "event timing");
        pf += a;
        st += b;
    }
    c->timed_from = c->k_host;
    if (ms_pf) *ms_pf = n > 0 ? pf / n : 0.0;
    if (ms_step) *ms_step = n > 0 ? st / n : 0.0;
    if (n_steps) *n_steps = n;
    return SMC2_OK;
}

extern "C" int smc2_info(smc2_ctx* c, int32_t run, int32_t k, smc2_step_info* info)
{
    if (!c) return g_thread_error = "ctx is NULL", SMC2_E_ARG;
    if (run < 0 || run >= c->R || !info) return c->fail(SMC2_E_ARG, "bad run or info");
    if (k < 1 || k > c->k_host) return c->fail(SMC2_E_ARG, "iteration k has not run");
    if (c->poisoned) return c->fail(SMC2_E_DEVICE, "context poisoned by an earlier device error");
    hipError_t e = hipStreamSynchronize(c->stream);
    const size_t RL = SMC2_RECORD_LEN(c->cfg.D);
    std::vector<double> rec(RL);
    unsigned long long at[2] = {0ull, 0ull};
    const unsigned long long* hist = c->oa.psteps_at + (size_t)run * c->cfg.K;
    if (e == hipSuccess)
        e = hipMemcpy(rec.data(), c->oa.records + ((size_t)run * c->cfg.K + (k - 1)) * RL, sizeof(double) * RL,
                      hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&at[1], hist + (k - 1), sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (e == hipSuccess && k > 1) e = hipMemcpy(&at[0], hist + (k - 2), sizeof(unsigned long long), hipMemcpyDeviceToHost);
    float t[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    const hipEvent_t* ev = &c->ev[EV_PER_STEP * (size_t)(k - 1)];
    if (e == hipSuccess) e = hipEventElapsedTime(&t[0], ev[0], ev[5]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t[1], ev[2], ev[3]);
    if (e == hipSuccess && !c->cfg.use_graph) {
        e = hipEventElapsedTime(&t[2], ev[0], ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&t[3], ev[1], ev[2]);
        if (e == hipSuccess) e = hipEventElapsedTime(&t[4], ev[3], ev[4]);
    }
    float t_train = 0.f;
    if (e == hipSuccess && !c->cfg.use_graph) e = hipEventElapsedTime(&t_train, ev[4], ev[5]);
    if (e != hipSuccess) return c->device_fail(e, "smc2_info");
    info->k = (int32_t)rec[0];
    info->ess = rec[1];
    info->resampled = (int32_t)rec[2];
    info->dead = (int32_t)rec[3];
    info->lkernel_fallback = (int32_t)rec[4];
    info->log_weight_sum = rec[5];
    info->proposal = (int32_t)rec[RL - 2];
    info->learned = info->proposal == 1 ? 1 : 0;
    info->particle_steps = at[1] - at[0];
    info->ms_step = t[0];
    info->ms_filters = t[1];
    if (c->cfg.use_graph) {
        info->ms_outer = -1.0;
        info->ms_mlp = -1.0;
    } else {
        // [0, 1): the learned proposal's forward pass (with the iteration's begin kernel),
        // [1, 2): the proposal, [3, 4): the outer update, [4, 5): training
        info->ms_outer = (double)t[3] + (double)t[4];
        info->ms_mlp = c->op.mlp ? (double)t[2] + (double)t_train : 0.0;
    }
    return SMC2_OK;
}

extern "C" int smc2_destroy(smc2_ctx* c)
{
    if (!c) return SMC2_OK;
    (void)hipStreamSynchronize(c->stream);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipEvent_t e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
    return SMC2_OK;
}

extern "C" const char* smc2_last_error(const smc2_ctx* c)
{
    if (c) return c->err.c_str();
    return g_thread_error.c_str();
}

extern "C" int smc2_groups(const smc2_ctx* c, int32_t max_groups, int32_t* n_groups, int32_t* desc, float* tuned_ms)
{
    if (!c || !n_groups) return g_thread_error = "ctx or n_groups is NULL", SMC2_E_ARG;
    *n_groups = (int32_t)c->groups.size();
    if (max_groups < 0 || (max_groups > 0 && !desc)) return g_thread_error = "bad desc buffer", SMC2_E_ARG;
    for (int g = 0; g < (int)c->groups.size() && g < max_groups; ++g) {
        const PFGroup& gr = c->groups[g];
        int32_t* d = desc + 6 * g;
        d[0] = gr.block;
        d[1] = (gr.sched == PF_SCHED_POOLED || gr.sched == PF_SCHED_SCORE_POOLED) ? SMC2_SCHED_POOLED
                                                                                 : SMC2_SCHED_PER_DRAW;
        d[2] = gr.persistent;
        d[3] = gr.persistent ? gr.grid : gr.n_items;
        d[4] = gr.n_items;
        d[5] = (int32_t)gr.lds;
        if (tuned_ms) tuned_ms[g] = gr.tuned_ms;
    }
    return SMC2_OK;
}

// ------------------------------------------------------------------ p-MCMC (Sec. III)

struct smc2_pmcmc {
    smc2_config cfg{};
    std::vector<double> prior, rw_cov, fixed;
    std::vector<int32_t> y;
    smc2_run run{};
    int C = 0, iters = 0, m_host = 0;
    unsigned char* ws = nullptr;
    hipStream_t stream = nullptr;
    McArrays ma{};
    McParams mp{};
    PFArgs pa{};
    int block = 0, sched = 0;
    size_t lds = 0;
    hipEvent_t ev_first = nullptr, ev_last = nullptr;
    bool timed = false, poisoned = false;
};

namespace {
struct McLayout {
    size_t total = 0;
    size_t off_run, off_y, off_prior, off_lrw, off_phi, off_lp, off_ll, off_phin, off_thn, off_lpn, off_lln, off_act,
        off_m, off_phit, off_llt, off_llnt, off_acct;
    size_t take(size_t bytes)
    {
        const size_t o = total;
        total += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

McLayout mc_layout(const smc2_config* c, int C, int iters, const smc2_run* run)
{
    McLayout L;
    const size_t D = (size_t)c->D;
    L.off_run = L.take(sizeof(RunDev));
    L.off_y = L.take(sizeof(int32_t) * (size_t)run->T * obs_words(c->model));
    L.off_prior = L.take(sizeof(double) * D * 3);
    L.off_lrw = L.take(sizeof(double) * D * D);
    L.off_phi = L.take(sizeof(double) * C * D);
    L.off_lp = L.take(sizeof(double) * C);
    L.off_ll = L.take(sizeof(double) * C);
    L.off_phin = L.take(sizeof(double) * C * D);
    L.off_thn = L.take(sizeof(double) * C * D);
    L.off_lpn = L.take(sizeof(double) * C);
    L.off_lln = L.take(sizeof(double) * C);
    L.off_act = L.take((size_t)C);
    L.off_m = L.take(sizeof(int32_t));
    L.off_phit = L.take(sizeof(double) * C * (size_t)(iters + 1) * D);
    L.off_llt = L.take(sizeof(double) * C * (size_t)(iters + 1));
    L.off_llnt = L.take(sizeof(double) * C * (size_t)iters);
    L.off_acct = L.take(sizeof(int32_t) * C * (size_t)iters);
    return L;
}

int mc_validate(const smc2_config* cfg, int32_t chains, int32_t iters, const smc2_run* run, std::string& m)
{
    if (!cfg || !run) return m = "null config or run", SMC2_E_ARG;
    if (chains < 1 || chains > 32768) return m = "chains must be in [1, 32768]", SMC2_E_ARG;
    if (iters < 0 || iters > 65535) return m = "iterations must be in [0, 65535]", SMC2_E_ARG;
    // the sampler's checks, with the population fields (unused here) set to valid values
    smc2_config c = *cfg;
    c.N = 2;
    c.K = 1;
    c.proposal = SMC2_PROP_RW;
    c.lkernel = SMC2_L_GAUSS_OPT;
    c.tune = 0;
    c.persistent = 0;
    c.mlp_train = SMC2_MLP_TRAIN_AUTO;
    return validate(&c, 1, run, m);
}

double host_theta_of(int fam, double v)
{
    if (fam == SMC2_PRIOR_LOGNORMAL) return std::exp(v);
    if (fam == SMC2_PRIOR_LOGITNORMAL) return 1.0 / (1.0 + std::exp(-v));
    return v;
}

hipError_t mc_filters(smc2_pmcmc* c)
{
    return launch_pf(c->cfg.precision, c->cfg.model, c->cfg.obs, c->sched, c->block, c->lds, c->pa, c->stream);
}
}  // namespace

extern "C" size_t smc2_pmcmc_workspace_bytes(const smc2_config* cfg, int32_t chains, int32_t iters, const smc2_run* run)
{
    std::string m;
    if (mc_validate(cfg, chains, iters, run, m) != SMC2_OK) {
        g_thread_error = m;
        return 0;
    }
    return mc_layout(cfg, chains, iters, run).total;
}

extern "C" int smc2_pmcmc_init(const smc2_config* cfg, int32_t chains, int32_t iters, const smc2_run* run,
                               void* d_workspace, size_t ws_bytes, void* hip_stream, smc2_pmcmc** out)
{
    if (!out) return g_thread_error = "out is NULL", SMC2_E_ARG;
    *out = nullptr;
    std::string m;
    int rc = mc_validate(cfg, chains, iters, run, m);
    if (rc != SMC2_OK) return g_thread_error = m, rc;
    const McLayout L = mc_layout(cfg, chains, iters, run);
    if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace & 255u))
        return g_thread_error = "workspace missing, too small or not 256-byte aligned", SMC2_E_ARG;
    const int block = cfg->block ? cfg->block : pf_default_block(cfg->model, cfg->precision, run->n_x, run->T, cfg->schedule);
    const int sched = pf_pick_schedule(cfg->model, cfg->precision, block, run->n_x, run->T, cfg->schedule);
    if (sched < 0) return g_thread_error = "the pooled schedule cannot run this model, n_x and T", SMC2_E_ARG;
    const size_t lds = pf_lds_bytes(cfg->model, cfg->precision, block, run->n_x, run->T, sched);
    if (lds > PF_LDS_MAX) return g_thread_error = "particle filter does not fit in LDS", SMC2_E_ARG;

    smc2_pmcmc* c = new smc2_pmcmc();
    c->cfg = *cfg;
    c->prior.assign(cfg->prior, cfg->prior + cfg->D * 3);
    c->rw_cov.assign(cfg->rw_cov, cfg->rw_cov + cfg->D * cfg->D);
    c->fixed.assign(SMC2_NFIXED, 0.0);
    for (int i = 0; i < cfg->n_fixed; ++i) c->fixed[i] = cfg->fixed[i];
    c->cfg.prior = c->prior.data();
    c->cfg.rw_cov = c->rw_cov.data();
    c->cfg.fixed = c->fixed.data();
    obs_pack(cfg->model, *run, c->y);
    c->run = *run;
    c->run.y = c->y.data();
    c->run.y_real = nullptr;
    c->C = chains;
    c->iters = iters;
    c->ws = (unsigned char*)d_workspace;
    c->stream = (hipStream_t)hip_stream;
    c->block = block;
    c->sched = sched;
    c->lds = lds;
    unsigned char* w = c->ws;
    McArrays& a = c->ma;
    a.phi = (double*)(w + L.off_phi);
    a.lp = (double*)(w + L.off_lp);
    a.ll = (double*)(w + L.off_ll);
    a.phi_new = (double*)(w + L.off_phin);
    a.theta_new = (double*)(w + L.off_thn);
    a.lp_new = (double*)(w + L.off_lpn);
    a.ll_new = (double*)(w + L.off_lln);
    a.active = (uint8_t*)(w + L.off_act);
    a.phi_trace = (double*)(w + L.off_phit);
    a.ll_trace = (double*)(w + L.off_llt);
    a.lln_trace = (double*)(w + L.off_llnt);
    a.acc_trace = (int32_t*)(w + L.off_acct);
    a.m_dev = (int32_t*)(w + L.off_m);
    McParams& p = c->mp;
    p.C = chains;
    p.D = cfg->D;
    p.iters = iters;
    p.prior = (const double*)(w + L.off_prior);
    p.lrw = (const double*)(w + L.off_lrw);
    PFArgs& f = c->pa;
    f.theta = a.theta_new;
    f.active = a.active;
    f.ll = a.ll_new;
    f.y = (const int32_t*)(w + L.off_y);
    f.runs = (const RunDev*)(w + L.off_run);
    f.items = nullptr;
    f.k_dev = a.m_dev;
    f.n_items = chains;
    f.N = chains;
    f.D = cfg->D;
    f.pf_always = cfg->pf_always;
    f.multinomial = cfg->pf_resampling;
    f.n_pop = cfg->n_pop;
    for (int i = 0; i < SMC2_NFIXED; ++i) f.fx[i] = c->fixed[i];

    std::vector<double> lrw((size_t)cfg->D * cfg->D);
    host_cholesky(cfg->D, cfg->rw_cov, lrw.data());
    const RunDev rd{run->T, run->n_x, 0, 0, (uint32_t)run->seed, (uint32_t)(run->seed >> 32)};
    hipStream_t s = c->stream;
    hipError_t e = hipMemcpyAsync(w + L.off_run, &rd, sizeof(rd), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w + L.off_y, c->y.data(), sizeof(int32_t) * c->y.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w + L.off_prior, c->prior.data(), sizeof(double) * c->prior.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w + L.off_lrw, lrw.data(), sizeof(double) * lrw.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.off_m, 0, sizeof(int32_t), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host copies above are released below
    // wave priorities when every chain's filter is resident at once
    int per_cu = 0, n_cu = 0, dev = 0;
    if (e == hipSuccess) e = pf_prepare(cfg->precision, cfg->model, cfg->obs, sched, lds);
    if (e == hipSuccess) e = pf_occupancy(cfg->precision, cfg->model, cfg->obs, sched, block, lds, &per_cu);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && (long)chains <= (long)per_cu * n_cu)
        f.prio_scale = (float)(1.0 / ((double)run->T * (double)run->n_x));
    if (e == hipSuccess) e = hipEventCreate(&c->ev_first);
    if (e == hipSuccess) e = hipEventCreate(&c->ev_last);
    // iteration 0: the chains' starting points and their filters
    if (e == hipSuccess) e = launch_mc_start(a, p, run->seed, s);
    if (e == hipSuccess) e = mc_filters(c);
    if (e == hipSuccess) e = launch_mc_accept(a, p, run->seed, s);
    if (e != hipSuccess) {
        g_thread_error = std::string("smc2_pmcmc_init: ") + hipGetErrorString(e);
        smc2_pmcmc_destroy(c);
        return SMC2_E_DEVICE;
    }
    *out = c;
    return SMC2_OK;
}

extern "C" int smc2_pmcmc_step(smc2_pmcmc* c, int32_t n_iter)
{
    if (!c) return g_thread_error = "ctx is NULL", SMC2_E_ARG;
    if (c->poisoned) return g_thread_error = "context poisoned by an earlier device error", SMC2_E_DEVICE;
    if (n_iter < 0) return g_thread_error = "n_iter < 0", SMC2_E_ARG;
    if (c->m_host + n_iter > c->iters) return g_thread_error = "more iterations than configured", SMC2_E_STATE;
    if (n_iter == 0) return SMC2_OK;
    hipError_t e = hipSuccess;
    if (!c->timed) e = hipEventRecord(c->ev_first, c->stream);
    for (int i = 0; i < n_iter && e == hipSuccess; ++i) {
        e = launch_mc_propose(c->ma, c->mp, c->run.seed, c->stream);
        if (e == hipSuccess) e = mc_filters(c);
        if (e == hipSuccess) e = launch_mc_accept(c->ma, c->mp, c->run.seed, c->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(c->ev_last, c->stream);
    if (e != hipSuccess) {
        c->poisoned = true;
        return g_thread_error = std::string("smc2_pmcmc_step: ") + hipGetErrorString(e), SMC2_E_DEVICE;
    }
    c->timed = true;
    c->m_host += n_iter;
    return SMC2_OK;
}

extern "C" int smc2_pmcmc_estimate(smc2_pmcmc* c, int32_t burn_in, double* mean, double* cov, double* accept_rate)
{
    if (!c || !mean) return g_thread_error = "ctx or mean is NULL", SMC2_E_ARG;
    if (burn_in < 0 || burn_in >= c->m_host) return g_thread_error = "burn_in must be in [0, iterations run)", SMC2_E_ARG;
    if (c->poisoned) return g_thread_error = "context poisoned by an earlier device error", SMC2_E_DEVICE;
    const int D = c->cfg.D, C = c->C, I = c->iters;
    std::vector<double> tr((size_t)C * (I + 1) * D);
    std::vector<int32_t> acc((size_t)C * (I > 0 ? I : 1));
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(tr.data(), c->ma.phi_trace, sizeof(double) * tr.size(), hipMemcpyDeviceToHost);
    if (e == hipSuccess && I > 0) e = hipMemcpy(acc.data(), c->ma.acc_trace, sizeof(int32_t) * C * I, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        c->poisoned = true;
        return g_thread_error = std::string("smc2_pmcmc_estimate: ") + hipGetErrorString(e), SMC2_E_DEVICE;
    }
    // mean and covariance of theta over the states after burn_in iterations, all chains
    std::vector<double> m(D, 0.0), S((size_t)D * D, 0.0);
    double n = 0.0, na = 0.0;
    for (int ch = 0; ch < C; ++ch)
        for (int it = burn_in + 1; it <= c->m_host; ++it) {
            double th[SMC2_DMAX];
            for (int d = 0; d < D; ++d)
                th[d] = host_theta_of((int)c->prior[3 * d], tr[((size_t)ch * (I + 1) + it) * D + d]);
            n += 1.0;
            for (int d = 0; d < D; ++d) m[d] += th[d];
            for (int d = 0; d < D; ++d)
                for (int f = 0; f < D; ++f) S[(size_t)d * D + f] += th[d] * th[f];
            na += acc[(size_t)ch * I + (it - 1)];
        }
    for (int d = 0; d < D; ++d) mean[d] = m[d] / n;
    if (cov)
        for (int d = 0; d < D; ++d)
            for (int f = 0; f < D; ++f) cov[(size_t)d * D + f] = S[(size_t)d * D + f] / n - mean[d] * mean[f];
    if (accept_rate) *accept_rate = na / n;
    return SMC2_OK;
}

extern "C" int smc2_pmcmc_dump(smc2_pmcmc* c, int32_t what, void* host_dst, size_t bytes)
{
    if (!c || !host_dst) return g_thread_error = "ctx or destination is NULL", SMC2_E_ARG;
    const size_t C = (size_t)c->C, I = (size_t)c->iters, D = (size_t)c->cfg.D;
    const void* src = nullptr;
    size_t need = 0;
    switch (what) {
    case SMC2_PMCMC_PHI: src = c->ma.phi_trace; need = C * (I + 1) * D * 8; break;
    case SMC2_PMCMC_LL: src = c->ma.ll_trace; need = C * (I + 1) * 8; break;
    case SMC2_PMCMC_LL_PROPOSED: src = c->ma.lln_trace; need = C * I * 8; break;
    case SMC2_PMCMC_ACCEPTED: src = c->ma.acc_trace; need = C * I * 4; break;
    default: return g_thread_error = "unknown dump", SMC2_E_ARG;
    }
    if (bytes < need) return g_thread_error = "destination too small", SMC2_E_ARG;
    if (c->poisoned) return g_thread_error = "context poisoned by an earlier device error", SMC2_E_DEVICE;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && need) e = hipMemcpy(host_dst, src, need, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        c->poisoned = true;
        return g_thread_error = std::string("smc2_pmcmc_dump: ") + hipGetErrorString(e), SMC2_E_DEVICE;
    }
    return SMC2_OK;
}

extern "C" int smc2_pmcmc_timing(smc2_pmcmc* c, double* ms, int32_t* iterations)
{
    if (!c) return g_thread_error = "ctx is NULL", SMC2_E_ARG;
    if (c->poisoned) return g_thread_error = "context poisoned by an earlier device error", SMC2_E_DEVICE;
    float t = 0.f;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && c->timed) e = hipEventElapsedTime(&t, c->ev_first, c->ev_last);
    if (e != hipSuccess) {
        c->poisoned = true;
        return g_thread_error = std::string("smc2_pmcmc_timing: ") + hipGetErrorString(e), SMC2_E_DEVICE;
    }
    if (ms) *ms = t;
    if (iterations) *iterations = c->m_host;
    return SMC2_OK;
}

extern "C" int smc2_pmcmc_destroy(smc2_pmcmc* c)
{
    if (!c) return SMC2_OK;
    (void)hipStreamSynchronize(c->stream);
    if (c->ev_first) (void)hipEventDestroy(c->ev_first);
    if (c->ev_last) (void)hipEventDestroy(c->ev_last);
    delete c;
    return SMC2_OK;
}
