// kernels_api.hip — kernel-level entry points (include/smc2_kernels.h): the
// building blocks of the sampler on caller-provided device arrays.
#include <mutex>
#include <string>
#include <vector>

#include "../../include/smc2_kernels.h"
#include "block_ops.h"
#include "mlp_kernels.h"
#include "obs_words.h"
#include "pf_kernel.h"

namespace smc2 {

__global__ void k_philox_batch(int n, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out)
{
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= n) return;
    const W4 w = philox10(ctr[4 * e], ctr[4 * e + 1], ctr[4 * e + 2], ctr[4 * e + 3], k0, k1);
    out[4 * e] = w.x;
    out[4 * e + 1] = w.y;
    out[4 * e + 2] = w.z;
    out[4 * e + 3] = w.w;
}

template <typename real>
__global__ void k_binomial_batch(int count, const int32_t* n, const double* p, uint32_t i, uint32_t kt, uint32_t b,
                                 uint32_t k0, uint32_t k1, int32_t* out)
{
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= count) return;
    out[j] = binomial<real>(n[j], (real)p[j], DrawStream{(uint32_t)j, i, kt, b, k0, k1});
}

__global__ void __launch_bounds__(256) k_resample_batch(int n, const uint64_t* q, const uint64_t* x64, int32_t* anc,
                                                        int32_t* trig)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ RedLds red;
    uint64_t* C = reinterpret_cast<uint64_t*>(smem);
    const int s = (int)blockIdx.x;
    const uint64_t* qs = q + (size_t)s * n;
    double dz = 0.0;
    uint64_t q1 = 0, q2 = 0;
    for (int j = (int)threadIdx.x; j < n; j += (int)blockDim.x) {
        const uint64_t v = qs[j];
        C[j] = v;
        const uint64_t h = v >> 8;
        q1 += h;
        q2 += h * h;
    }
    block_sum3(dz, q1, q2, &red);
    const uint64_t Q = block_scan_lds(C, n, &red);
    block_ancestors(C, n, Q, x64[s], anc + (size_t)s * n);
    if (threadIdx.x == 0) trig[s] = ess_below_half(q1, q2, n) ? 1 : 0;
}

}  // namespace smc2

// Scratch of smc2_pf_loglik_noalloc: the run descriptor (256 bytes) and the observation
// series (at most 1024 days x 4 series x 4 bytes), the contents of smc2_pf_loglik's
// workspace. Host code never names it in a copy or a launch: in host code the name is
// a host-side stand-in; pf_static_scratch() gives the device address.
#define PF_STATIC_SCRATCH_BYTES (256 + 1024 * 4 * 4)
static __device__ __align__(256) unsigned char scratch[PF_STATIC_SCRATCH_BYTES];

using namespace smc2;

// defined in smc2_api.cpp: the thread's message for smc2_last_error(NULL)
void smc2_set_thread_error(const std::string& m);

namespace {
int kfail(int code, const std::string& m)
{
    smc2_set_thread_error(m);
    return code;
}

// Device address of `scratch` on the current device, resolved with that device current
// on the first call there and kept per device (each device holds its own copy).
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES];

hipError_t pf_static_scratch(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

extern "C" int smc2_philox_batch(int32_t n, const uint32_t* d_ctr, uint64_t seed, uint32_t* d_out, void* stream)
{
    if (n < 0 || (n > 0 && (!d_ctr || !d_out))) return kfail(SMC2_E_ARG, "bad philox arguments");
    if (n == 0) return SMC2_OK;
    hipLaunchKernelGGL(k_philox_batch, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n, d_ctr,
                       (uint32_t)seed, (uint32_t)(seed >> 32), d_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SMC2_OK : kfail(SMC2_E_DEVICE, hipGetErrorString(e));
}

extern "C" int smc2_binomial_batch(int32_t precision, int32_t count, const int32_t* d_n, const double* d_p,
                                   uint64_t seed, uint32_t i, uint32_t k, uint32_t t, uint32_t b, int32_t* d_out,
                                   void* stream)
{
    if (count < 0 || (count > 0 && (!d_n || !d_p || !d_out))) return kfail(SMC2_E_ARG, "bad binomial arguments");
    if (precision != SMC2_PREC_FP32 && precision != SMC2_PREC_FP64) return kfail(SMC2_E_ARG, "bad precision");
    if (k > 65535 || t > 65535 || b > 255) return kfail(SMC2_E_ARG, "k, t or b out of range");
    if (count == 0) return SMC2_OK;
    const dim3 g((unsigned)((count + 255) / 256)), blk(256);
    const uint32_t kt = (k << 16) | t, k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (precision == SMC2_PREC_FP32)
        hipLaunchKernelGGL(k_binomial_batch<float>, g, blk, 0, (hipStream_t)stream, count, d_n, d_p, i, kt, b, k0, k1,
                           d_out);
    else
        hipLaunchKernelGGL(k_binomial_batch<double>, g, blk, 0, (hipStream_t)stream, count, d_n, d_p, i, kt, b, k0, k1,
                           d_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SMC2_OK : kfail(SMC2_E_DEVICE, hipGetErrorString(e));
}

extern "C" int smc2_resample_batch(int32_t n_sets, int32_t n, const uint64_t* d_q, const uint64_t* d_x64,
                                   int32_t* d_anc, int32_t* d_trigger, void* stream)
{
    if (n_sets < 0 || n < 1 || n > 4096) return kfail(SMC2_E_ARG, "n must be in [1, 4096]");
    if (n_sets > 0 && (!d_q || !d_x64 || !d_anc || !d_trigger)) return kfail(SMC2_E_ARG, "null pointer");
    if (n_sets == 0) return SMC2_OK;
    hipLaunchKernelGGL(k_resample_batch, dim3((unsigned)n_sets), dim3(256), (size_t)n * 8, (hipStream_t)stream, n,
                       d_q, d_x64, d_anc, d_trigger);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SMC2_OK : kfail(SMC2_E_DEVICE, hipGetErrorString(e));
}

extern "C" size_t smc2_pf_workspace_bytes(const smc2_config* cfg, const smc2_run* run)
{
    if (!cfg || !run || run->T < 1) {
        kfail(SMC2_E_ARG, "cfg or run is NULL, or run->T < 1");
        return 0;
    }
    const size_t y = ((size_t)run->T * obs_words(cfg->model) * 4 + 255) & ~(size_t)255;
    return 256 + y;
}

extern "C" int smc2_pf_loglik(const smc2_config* cfg, int32_t n_theta, const double* d_theta, const smc2_run* run,
                              uint32_t k, double* d_ll, void* d_ws, size_t ws_bytes, void* stream)
{
    return smc2_pf_trace(cfg, n_theta, d_theta, run, k, d_ll, nullptr, nullptr, d_ws, ws_bytes, stream);
}

static int pf_run(const smc2_config* cfg, int32_t n_theta, const double* d_theta, const smc2_run* run, uint32_t k,
                  double* d_ll, double* d_inc, int32_t* d_rs, int32_t* d_state, int32_t* d_anc, double* d_score,
                  void* d_ws, size_t ws_bytes, void* stream, bool static_ws = false, bool score = false);

extern "C" int smc2_pf_trace(const smc2_config* cfg, int32_t n_theta, const double* d_theta, const smc2_run* run,
                             uint32_t k, double* d_ll, double* d_inc, int32_t* d_rs, void* d_ws, size_t ws_bytes,
                             void* stream)
{
    return pf_run(cfg, n_theta, d_theta, run, k, d_ll, d_inc, d_rs, nullptr, nullptr, nullptr, d_ws, ws_bytes, stream);
}

extern "C" int smc2_pf_trace_state(const smc2_config* cfg, int32_t n_theta, const double* d_theta,
                                   const smc2_run* run, uint32_t k, double* d_ll, double* d_inc, int32_t* d_rs,
                                   int32_t* d_state, int32_t* d_anc, void* d_ws, size_t ws_bytes, void* stream)
{
    if (!d_state) return kfail(SMC2_E_ARG, "d_state is NULL");
    return pf_run(cfg, n_theta, d_theta, run, k, d_ll, d_inc, d_rs, d_state, d_anc, nullptr, d_ws, ws_bytes, stream);
}

extern "C" int smc2_pf_score(const smc2_config* cfg, int32_t n_theta, const double* d_theta, const smc2_run* run,
                             uint32_t k, double* d_ll, double* d_score, void* d_ws, size_t ws_bytes, void* stream)
{
    if (n_theta > 0 && !d_score) return kfail(SMC2_E_ARG, "d_score is NULL");
    if (!cfg) return kfail(SMC2_E_ARG, "null config or run");
    if (pf_score_dims(cfg->model) == 0) return kfail(SMC2_E_UNSUPPORTED, "no score for this model");
    if (cfg->model == SMC2_SEIR && cfg->D != 4 && cfg->D != 5) return kfail(SMC2_E_ARG, "SEIR needs D = 4 or 5");
    if (cfg->model != SMC2_SEIR && cfg->D != pf_score_dims(cfg->model)) return kfail(SMC2_E_ARG, "bad D");
    return pf_run(cfg, n_theta, d_theta, run, k, d_ll, nullptr, nullptr, nullptr, nullptr, d_score, d_ws, ws_bytes,
                  stream, false, true);
}

extern "C" int smc2_pf_loglik_noalloc(const smc2_config* cfg, int32_t n_theta, const double* d_theta,
                                      const smc2_run* run, uint32_t k, double* d_ll, void* stream)
{
    return pf_run(cfg, n_theta, d_theta, run, k, d_ll, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, stream,
                  true);
}

// static_ws: the workspace is the file-scope scratch (d_ws and ws_bytes unused); its
// device address is resolved only after every argument has been checked.
// score: the score launch into d_score (the per-draw schedule carrying each particle's score)
static int pf_run(const smc2_config* cfg, int32_t n_theta, const double* d_theta, const smc2_run* run, uint32_t k,
                  double* d_ll, double* d_inc, int32_t* d_rs, int32_t* d_state, int32_t* d_anc, double* d_score,
                  void* d_ws, size_t ws_bytes, void* stream, bool static_ws, bool score)
{
    if ((d_inc == nullptr) != (d_rs == nullptr)) return kfail(SMC2_E_ARG, "trace needs both d_inc and d_rs");
    if (!cfg || !run) return kfail(SMC2_E_ARG, "null config or run");
    if (!pf_supported(cfg->model, cfg->obs)) return kfail(SMC2_E_UNSUPPORTED, "model/observation not supported");
    if (cfg->precision != SMC2_PREC_FP32 && cfg->precision != SMC2_PREC_FP64) return kfail(SMC2_E_ARG, "precision");
    const bool lg = cfg->model == SMC2_LINGAUSS;
    if (lg && cfg->precision != SMC2_PREC_FP64)
        return kfail(SMC2_E_UNSUPPORTED, "the linear-Gaussian model runs in FP64 only");
    if (cfg->D < 1 || cfg->D > SMC2_DMAX || (lg && cfg->D != 3)) return kfail(SMC2_E_ARG, "bad D");
    if (run->T < 1 || run->T > 1024 || run->n_x < 1 || run->n_x > (cfg->model == SMC2_AGE_SEIR ? 2048 : 4096))
        return kfail(SMC2_E_ARG, "T or n_x out of range");
    if (!lg && !(cfg->n_pop >= 1.0 && cfg->n_pop <= 16777216.0)) return kfail(SMC2_E_ARG, "n_pop out of range");
    if (k > 65535) return kfail(SMC2_E_ARG, "k out of range");
    if (cfg->pf_resampling != SMC2_PF_RS_SYSTEMATIC && cfg->pf_resampling != SMC2_PF_RS_MULTINOMIAL)
        return kfail(SMC2_E_ARG, "pf_resampling must be SMC2_PF_RS_SYSTEMATIC or SMC2_PF_RS_MULTINOMIAL");
    if (n_theta < 0 || (n_theta > 0 && (!d_theta || !d_ll))) return kfail(SMC2_E_ARG, "bad theta/ll");
    if (static_ws) {
        const size_t need = smc2_pf_workspace_bytes(cfg, run);
        if (need > PF_STATIC_SCRATCH_BYTES)
            return kfail(SMC2_E_ARG, "run needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                                         std::to_string(PF_STATIC_SCRATCH_BYTES));
    } else if (!d_ws || ws_bytes < smc2_pf_workspace_bytes(cfg, run) || ((uintptr_t)d_ws & 255u)) {
        return kfail(SMC2_E_ARG, "workspace missing, too small or not 256-byte aligned");
    }
    if (cfg->n_fixed < 0 || cfg->n_fixed > SMC2_NFIXED || (cfg->n_fixed > 0 && !cfg->fixed))
        return kfail(SMC2_E_ARG, "bad fixed constants");
    if (const char* why = obs_check(cfg->model, *run)) return kfail(SMC2_E_ARG, why);
    if (cfg->block != 0 && (cfg->block < 64 || cfg->block > 1024 || cfg->block % 64 != 0))
        return kfail(SMC2_E_ARG, "block must be 0 or a multiple of 64 up to 1024");
    if (cfg->schedule < 0 || cfg->schedule > 2) return kfail(SMC2_E_ARG, "schedule must be 0, 1 or 2");
    const int want = cfg->schedule;
    const int block =
        cfg->block ? cfg->block : pf_default_block(cfg->model, cfg->precision, run->n_x, run->T, want, score);
    const int sched = pf_pick_schedule(cfg->model, cfg->precision, block, run->n_x, run->T, want, score);
    if (sched < 0) return kfail(SMC2_E_ARG, "the pooled schedule cannot run this model, n_x and T");
    const size_t lds = pf_lds_bytes(cfg->model, cfg->precision, block, run->n_x, run->T, sched);
    if (lds > PF_LDS_MAX) return kfail(SMC2_E_ARG, "particle filter does not fit in LDS");
    if (n_theta == 0) return SMC2_OK;
    if (static_ws) {
        const hipError_t es = pf_static_scratch(&d_ws);
        if (es != hipSuccess) return kfail(SMC2_E_DEVICE, hipGetErrorString(es));
    }
    hipStream_t s = (hipStream_t)stream;
    unsigned char* w = (unsigned char*)d_ws;
    // every argument is checked before the first copy: from here on the host copies of rd
    // and the observation words must stay valid until the stream has run the copies, also
    // on a device error (the stream is synchronised before returning)
    std::vector<int32_t> yw;
    obs_pack(cfg->model, *run, yw);
    RunDev rd{run->T, run->n_x, 0, 0, (uint32_t)run->seed, (uint32_t)(run->seed >> 32)};
    hipError_t e = hipMemcpyAsync(w, &rd, sizeof(rd), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w + 256, yw.data(), yw.size() * 4, hipMemcpyHostToDevice, s);
    PFArgs a{};
    a.theta = d_theta;
    a.active = nullptr;
    a.ll = d_ll;
    a.y = (const int32_t*)(w + 256);
    a.runs = (const RunDev*)w;
    a.items = nullptr;
    a.k_dev = nullptr;
    a.trace_inc = d_inc;
    a.trace_rs = d_rs;
    a.trace_state = d_state;
    a.trace_anc = d_anc;
    a.score = d_score;
    a.k_const = k;
    a.n_items = n_theta;
    a.N = n_theta;
    a.D = cfg->D;
    a.pf_always = cfg->pf_always;
    a.multinomial = cfg->pf_resampling;
    a.n_pop = cfg->n_pop;
    for (int i = 0; i < SMC2_NFIXED; ++i) a.fx[i] = i < cfg->n_fixed ? cfg->fixed[i] : 0.0;
    if (e == hipSuccess) e = pf_prepare(cfg->precision, cfg->model, cfg->obs, sched, lds);
    // wave priorities when every filter is resident at once (they even out its tail)
    int per_cu = 0, n_cu = 0, dev = 0;
    if (e == hipSuccess) e = pf_occupancy(cfg->precision, cfg->model, cfg->obs, sched, block, lds, &per_cu);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && (long)n_theta <= (long)per_cu * n_cu)
        a.prio_scale = (float)(1.0 / ((double)run->T * (double)run->n_x));
    if (e == hipSuccess) e = launch_pf(cfg->precision, cfg->model, cfg->obs, sched, block, lds, a, s);
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    return e == hipSuccess ? SMC2_OK : kfail(SMC2_E_DEVICE, hipGetErrorString(e));
}

extern "C" int smc2_mlp_forward(int32_t D, int32_t n, const float* d_params, const double* d_frame, const double* d_phi,
                                float* d_out, void* stream)
{
    if (D < 1 || D > 8 || n < 0) return kfail(SMC2_E_ARG, "D must be in [1, 8] and n >= 0");
    if (n > 0 && (!d_params || !d_frame || !d_phi || !d_out)) return kfail(SMC2_E_ARG, "null pointer");
    hipError_t e = mlp_prepare(D);
    if (e == hipSuccess) e = launch_mlp_rows_forward(D, n, d_params, d_frame, d_phi, d_out, (hipStream_t)stream);
    return e == hipSuccess ? SMC2_OK : kfail(SMC2_E_DEVICE, hipGetErrorString(e));
}

extern "C" int smc2_mlp_grad(int32_t D, int32_t n, const float* d_params, const double* d_frame, const double* d_phi_in,
                             const double* d_phi_t, const double* d_w, float* d_grad, double* d_loss, void* stream)
{
    if (D < 1 || D > 8 || n < 1 || n > 32768) return kfail(SMC2_E_ARG, "D must be in [1, 8] and n in [1, 32768]");
    if (!d_params || !d_frame || !d_phi_in || !d_phi_t || !d_w || !d_grad || !d_loss)
        return kfail(SMC2_E_ARG, "null pointer");
    hipError_t e = mlp_prepare(D);
    if (e == hipSuccess)
        e = launch_mlp_rows_grad(D, n, d_params, d_frame, d_phi_in, d_phi_t, d_w, d_grad, d_loss, (hipStream_t)stream);
    return e == hipSuccess ? SMC2_OK : kfail(SMC2_E_DEVICE, hipGetErrorString(e));
}
