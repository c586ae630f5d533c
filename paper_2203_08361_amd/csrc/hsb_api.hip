// libhsb C ABI: argument validation, the J store, run orchestration.
// Declarations and the contract of every entry point are in include/hsb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "batch.h"
#include "digits.h"
#include "hsb.h"
#include "kernels.h"
#include "persistent.h"
#include "tune.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? HSB_ENOMEM : HSB_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return hip_fail(_e, #expr); \
    } while (0)

inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

// FP4 (E2M1) values: 0, 0.5, 1, 1.5, 2, 3, 4, 6 and their negatives.
bool fp4_exact(float v) {
    const float a = std::fabs(v);
    return a == 0.0f || a == 0.5f || a == 1.0f || a == 1.5f || a == 2.0f || a == 3.0f ||
           a == 4.0f || a == 6.0f;
}

}  // namespace

// Work space of hsb_run_ex_noalloc: one fixed array per device, held from the
// library's first use of the device until the process ends.  Host code never
// passes this name to a kernel (on the host it is only a stand-in for the
// device symbol): it uses the address hipGetSymbolAddress returns per device.
static __device__ __align__(256) unsigned char scratch[HSB_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current (looked up
// once per device, at the first context created on it).
int scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices)
        return fail(HSB_EDEVICE, "device %d beyond the %d the library supports", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(HSB_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return HSB_OK;
}

__global__ void k_flag_clear(int32_t *flag) { flag[0] = 0; }

// flag = 1 if some gamma_rep[r], r < R, is not finite or is negative
__global__ void k_flag_bad_gamma(const float *__restrict__ g, int R, int32_t *flag) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R && !(isfinite(g[r]) && g[r] >= 0.0f)) atomicOr(flag, 1);
}

}  // namespace

struct hsb_ctx {
    int N = 0, Npad = 0, device = 0;
    float *dJ = nullptr;        // FP32 J, [Npad][Npad], zero padded
    bool j_int_exact = false;   // integer J with small row sums: FP32 fields exact
    bool j_fp4_exact = false;   // every entry representable in FP4 (E2M1)
    bool j_i8_exact = false;    // every entry an integer in [-127, 127]
    hsb::PersistentJ *pj = nullptr;  // FP4 J store for the persistent dSB path (lazy)
    hsb::I8J *i8 = nullptr;          // integer-digit J store (lazy)
    hsb::PersistentWork *bwork = nullptr;  // scratch of batched FP4 runs led by this context
    hsb::QueueWork *qwork = nullptr;       // tables and buffers of queued dSB batches it leads
    // graph of the last repeated queued batch led by this context
    std::vector<uint64_t> bgkey;
    bool bgseen = false;
    hipGraphExec_t bgexec = nullptr;
    hsb::StateBufs bstate{};               // state of batch classes led by this context
    size_t bstate_ns = 0, bstate_nr = 0;   // its capacity: elements, columns
    hsb::BatchJob *bjobs = nullptr;        // device job table of a batch class
    size_t bjobs_cap = 0;
    int32_t *d_flag = nullptr;             // start-state bound check
    hsb::NHState nh{};                     // thermostat of the current run
    hsb::IncState inc{};                   // incremental dSB field
    size_t inc_cap = 0;                    // its capacity in Rpad * Npad elements
    int nh_cap = 0;                        // its capacity in columns
    std::vector<float> hJ;      // host copy kept for lazy device re-layouts
    // options
    double init_amp = 0.1;
    int interval = 100;
    int return_best = 1;
    int precision = HSB_PREC_AUTO;
    int timing = 0;
    int last_plan = -1;
    int local_exchange = 1;
    int graph = 1;
    int autotune = 0;   // HSB_OPT_AUTOTUNE
    int tile = -1;      // HSB_OPT_TILE: -1 default / tuned, else a forced variant
    int last_tile = 0;  // variant of the last successful run
    hsb::KernelTimer timer;
    // graph of the last repeated run (HSB_OPT_GRAPH): the key of that run, whether
    // it ran once eagerly, the instantiated graph, its stream and the events that
    // order it after and before the caller's stream
    std::vector<uint64_t> gkey;
    bool gseen = false;
    hipGraphExec_t gexec = nullptr;
    hipStream_t gstream = nullptr;
    hipEvent_t gev_in = nullptr, gev_out = nullptr;
    uint64_t glaunches = 0;
    // the run's seed: pinned host slot written by every call, device copy read by
    // the initialiser (a graph launch then takes the seed of its call)
    uint64_t *h_seed = nullptr;
    uint64_t *d_seed = nullptr;
    // cancellation: the request (pinned host word and its device view), the
    // per-step plans' stop word, and whether runs of this context poll it
    int32_t *h_cancel = nullptr;
    const int32_t *d_cancel = nullptr;
    int32_t *d_stop = nullptr;
    bool cancellable = true;  // false while a batch runs its jobs through hsb_run_ex
    int cancel_opt = 0;       // HSB_OPT_CANCELLABLE
    // workspace
    int Rpad_cap = 0;
    uint64_t state_gen = 0;  // raised when the state buffers are reallocated
    hsb::StateBufs b{};
    int8_t *d_spins = nullptr;  // hsb_run staging
    double *d_energy = nullptr;
    size_t run_cap = 0;
    hipStream_t stream = nullptr;
};

namespace {

void free_state(hsb_ctx *h) {
    hsb::free_state_bufs(h->b);
    h->Rpad_cap = 0;
}

int ensure_state(hsb_ctx *h, int Rpad) {
    if (Rpad <= h->Rpad_cap) return HSB_OK;
    free_state(h);
    ++h->state_gen;
    hipError_t e = hsb::alloc_state(h->b, h->Npad, Rpad);
    if (e != hipSuccess) return hip_fail(e, "allocating run state");
    h->Rpad_cap = Rpad;
    return HSB_OK;
}

bool finite_f(float v) { return std::isfinite(v); }

void graph_drop(hsb_ctx *h) {
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
    h->gseen = false;
    h->gkey.clear();
}

void batch_graph_drop(hsb_ctx *h) {
    if (h->bgexec) (void)hipGraphExecDestroy(h->bgexec);
    h->bgexec = nullptr;
    h->bgseen = false;
    h->bgkey.clear();
}

}  // namespace

// --------------------------------------------------------------------- API

extern "C" const char *hsb_last_error(void) { return g_err; }

extern "C" int hsb_cancel(hsb_ctx *h) {
    if (!h || !h->h_cancel) return fail(HSB_EINVAL, "hsb_cancel: NULL context");
    if (!__atomic_load_n(&h->cancel_opt, __ATOMIC_RELAXED))
        return fail(HSB_EINVAL, "hsb_cancel: the context's runs are not cancellable "
                                "(HSB_OPT_CANCELLABLE = 0)");
    __atomic_store_n(h->h_cancel, 1, __ATOMIC_SEQ_CST);
    return HSB_OK;
}

extern "C" int hsb_create(const float *J, int N, hsb_ctx **out) {
    g_err[0] = 0;
    if (!out) return fail(HSB_EINVAL, "hsb_create: out is NULL");
    *out = nullptr;
    if (!J) return fail(HSB_EINVAL, "hsb_create: J is NULL");
    if (N < 1 || N > 32768) return fail(HSB_EINVAL, "hsb_create: N=%d outside [1, 32768]", N);
    bool is_int = true, is_fp4 = true, is_i8 = true;
    double max_row = 0.0;
    for (int i = 0; i < N; ++i) {
        double row = 0.0;
        for (int j = 0; j < N; ++j) {
            const float v = J[(size_t)i * N + j];
            if (!finite_f(v)) return fail(HSB_EINVAL, "hsb_create: J[%d][%d] is not finite", i, j);
            if (v != J[(size_t)j * N + i])
                return fail(HSB_EINVAL, "hsb_create: J is not symmetric at (%d, %d)", i, j);
            if (i == j && v != 0.0f)
                return fail(HSB_EINVAL, "hsb_create: J[%d][%d] = %g, diagonal must be 0", i, i, v);
            if (v != std::nearbyint(v)) is_int = false;
            if (!fp4_exact(v)) is_fp4 = false;
            if (v != std::nearbyint(v) || std::fabs(v) > 127.0f) is_i8 = false;
            row += std::fabs((double)v);
        }
        if (row > max_row) max_row = row;
    }
    int dev = 0, ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(HSB_EDEVICE, "hsb_create: no HIP device");
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(HSB_EDEVICE, "hsb_create: device %d is %s, libhsb is built for gfx950", dev,
                    prop.gcnArchName);

    hsb_ctx *h = new (std::nothrow) hsb_ctx;
    if (!h) return fail(HSB_ENOMEM, "hsb_create: host allocation failed");
    h->N = N;
    h->Npad = round_up(N, hsb::kTile);
    h->device = dev;
    // integer products/sums stay below 2^24 in FP32 (32-row partial energies included)
    h->j_int_exact = is_int && max_row * 32.0 < 16777216.0;
    h->j_fp4_exact = is_fp4;
    h->j_i8_exact = is_i8;
    const size_t np = (size_t)h->Npad;
    std::vector<float> padded(np * np, 0.0f);
    for (int i = 0; i < N; ++i)
        std::memcpy(&padded[(size_t)i * np], J + (size_t)i * N, sizeof(float) * N);
    hipError_t e = hipMalloc((void **)&h->dJ, np * np * sizeof(float));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipMemcpy(h->dJ, padded.data(), np * np * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&h->h_cancel, sizeof(int32_t),
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
        *h->h_cancel = 0;
        void *dv = nullptr;
        e = hipHostGetDevicePointer(&dv, h->h_cancel, 0);
        h->d_cancel = static_cast<const int32_t *>(dv);
    }
    if (e == hipSuccess) e = hipMalloc((void **)&h->d_stop, sizeof(int32_t));
    if (e != hipSuccess) {
        int rc = hip_fail(e, "hsb_create: J store");
        hsb_destroy(h);
        return rc;
    }
    h->hJ.assign(J, J + (size_t)N * N);
    // the FP4 J store is built here when it applies, so that a run never has
    // to allocate it (hsb_run_ex_noalloc relies on that)
    if (h->j_fp4_exact && hsb::persistent_supported(N)) {
        const int rc = hsb::persistent_create(h->hJ.data(), N, &h->pj);
        if (rc != HSB_OK) {
            fail(rc, "hsb_create: %s", hsb::persistent_error());
            hsb_destroy(h);
            return rc;
        }
    }
    void *scr = nullptr;
    const int rc = scratch_address(dev, &scr);
    if (rc != HSB_OK) {
        hsb_destroy(h);
        return rc;
    }
    *out = h;
    return HSB_OK;
}

extern "C" void hsb_destroy(hsb_ctx *h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_state(h);
    if (h->dJ) (void)hipFree(h->dJ);
    if (h->d_spins) (void)hipFree(h->d_spins);
    if (h->d_energy) (void)hipFree(h->d_energy);
    if (h->pj) hsb::persistent_free(h->pj);
    if (h->i8) hsb::i8_free(h->i8);
    if (h->bwork) hsb::persistent_work_free(h->bwork);
    batch_graph_drop(h);
    if (h->qwork) hsb::queue_work_free(h->qwork);
    hsb::free_state_bufs(h->bstate);
    if (h->bjobs) (void)hipFree(h->bjobs);
    if (h->d_flag) (void)hipFree(h->d_flag);
    if (h->nh.xi) (void)hipFree(h->nh.xi);
    if (h->nh.part) (void)hipFree(h->nh.part);
    if (h->inc.F) (void)hipFree(h->inc.F);
    if (h->inc.list) (void)hipFree(h->inc.list);
    if (h->inc.cnt) (void)hipFree(h->inc.cnt);
    graph_drop(h);
    if (h->gev_in) (void)hipEventDestroy(h->gev_in);
    if (h->gev_out) (void)hipEventDestroy(h->gev_out);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    if (h->h_seed) (void)hipHostFree(h->h_seed);
    if (h->d_seed) (void)hipFree(h->d_seed);
    if (h->h_cancel) (void)hipHostFree(h->h_cancel);
    if (h->d_stop) (void)hipFree(h->d_stop);
    h->timer.release();
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

extern "C" int hsb_set_option(hsb_ctx *h, int key, double v) {
    if (!h) return fail(HSB_EINVAL, "hsb_set_option: NULL context");
    switch (key) {
    case HSB_OPT_INIT_AMP:
        if (!(std::isfinite(v) && v > 0.0 && v <= 1.0e6))
            return fail(HSB_EINVAL, "INIT_AMP must be finite and > 0");
        h->init_amp = v;
        return HSB_OK;
    case HSB_OPT_ENERGY_INTERVAL:
        if (!(v >= 1.0 && v <= 2147483647.0 && v == std::floor(v)))
            return fail(HSB_EINVAL, "ENERGY_INTERVAL must be an integer >= 1");
        h->interval = (int)v;
        return HSB_OK;
    case HSB_OPT_RETURN_BEST:
        if (!(v == 0.0 || v == 1.0)) return fail(HSB_EINVAL, "RETURN_BEST must be 0 or 1");
        h->return_best = (int)v;
        return HSB_OK;
    case HSB_OPT_PRECISION:
        if (!(v == HSB_PREC_AUTO || v == HSB_PREC_FP32 || v == HSB_PREC_MIXED ||
              v == HSB_PREC_DIGITS || v == HSB_PREC_INCREMENTAL))
            return fail(HSB_EINVAL, "PRECISION must be AUTO (0), FP32 (1), MIXED (2), DIGITS (3) "
                                    "or INCREMENTAL (4)");
        h->precision = (int)v;
        return HSB_OK;
    case HSB_OPT_TIMING:
        if (!(v == 0.0 || v == 1.0)) return fail(HSB_EINVAL, "TIMING must be 0 or 1");
        h->timing = (int)v;
        return HSB_OK;
    case HSB_OPT_LOCAL_EXCHANGE:
        if (!(v == 0.0 || v == 1.0)) return fail(HSB_EINVAL, "LOCAL_EXCHANGE must be 0 or 1");
        h->local_exchange = (int)v;
        return HSB_OK;
    case HSB_OPT_GRAPH:
        if (!(v == 0.0 || v == 1.0)) return fail(HSB_EINVAL, "GRAPH must be 0 or 1");
        h->graph = (int)v;
        if (!h->graph) {
            graph_drop(h);
            batch_graph_drop(h);
        }
        return HSB_OK;
    case HSB_OPT_AUTOTUNE:
        if (!(v == 0.0 || v == 1.0)) return fail(HSB_EINVAL, "AUTOTUNE must be 0 or 1");
        h->autotune = (int)v;
        return HSB_OK;
    case HSB_OPT_TILE:
        if (!(v == std::floor(v) && v >= -1.0 && v <= 15.0))
            return fail(HSB_EINVAL, "TILE must be -1 or a variant index 0 .. 15");
        h->tile = (int)v;
        return HSB_OK;
    case HSB_OPT_CANCELLABLE:
        if (!(v == 0.0 || v == 1.0)) return fail(HSB_EINVAL, "CANCELLABLE must be 0 or 1");
        __atomic_store_n(&h->cancel_opt, (int)v, __ATOMIC_RELAXED);
        return HSB_OK;
    case HSB_OPT_KERNEL_MS:
    case HSB_OPT_KERNEL_LAUNCHES:
    case HSB_OPT_LAST_PLAN:
    case HSB_OPT_GRAPH_LAUNCHES:
    case HSB_OPT_LAST_TILE:
        return fail(HSB_EINVAL, "option %d is read only", key);
    default:
        return fail(HSB_EINVAL, "unknown option key %d", key);
    }
}

extern "C" int hsb_get_option(hsb_ctx *h, int key, double *v) {
    if (!h || !v) return fail(HSB_EINVAL, "hsb_get_option: NULL argument");
    switch (key) {
    case HSB_OPT_INIT_AMP: *v = h->init_amp; return HSB_OK;
    case HSB_OPT_ENERGY_INTERVAL: *v = h->interval; return HSB_OK;
    case HSB_OPT_RETURN_BEST: *v = h->return_best; return HSB_OK;
    case HSB_OPT_PRECISION: *v = h->precision; return HSB_OK;
    case HSB_OPT_TIMING: *v = h->timing; return HSB_OK;
    case HSB_OPT_KERNEL_MS: {
        double ms = 0.0;
        hipError_t e = h->timer.total_ms(&ms);
        if (e != hipSuccess) return hip_fail(e, "reading kernel timing events");
        *v = ms;
        return HSB_OK;
    }
    case HSB_OPT_KERNEL_LAUNCHES: *v = (double)h->timer.launches; return HSB_OK;
    case HSB_OPT_LAST_PLAN: *v = h->last_plan; return HSB_OK;
    case HSB_OPT_LOCAL_EXCHANGE: *v = h->local_exchange; return HSB_OK;
    case HSB_OPT_GRAPH: *v = h->graph; return HSB_OK;
    case HSB_OPT_GRAPH_LAUNCHES: *v = (double)h->glaunches; return HSB_OK;
    case HSB_OPT_AUTOTUNE: *v = h->autotune; return HSB_OK;
    case HSB_OPT_TILE: *v = h->tile; return HSB_OK;
    case HSB_OPT_LAST_TILE: *v = h->last_tile; return HSB_OK;
    case HSB_OPT_CANCELLABLE: *v = h->cancel_opt; return HSB_OK;
    default: return fail(HSB_EINVAL, "unknown option key %d", key);
    }
}

extern "C" int hsb_num_samples(hsb_ctx *h, int start_step, int steps, int *n) {
    if (!h || !n) return fail(HSB_EINVAL, "hsb_num_samples: NULL argument");
    if (start_step < 0 || steps < 0 || (long long)start_step + steps > INT32_MAX)
        return fail(HSB_EINVAL, "hsb_num_samples: start_step and steps must be >= 0");
    const int I = h->interval, k1 = start_step + steps;
    *n = k1 / I - start_step / I + ((k1 % I != 0 || steps == 0) ? 1 : 0);
    return HSB_OK;
}

namespace {

// Execution plans (hsb_plan); the precision reported for both mixed plans is
// HSB_PREC_MIXED.
enum Plan {
    PLAN_FP32 = HSB_PLAN_FP32,
    PLAN_FP4 = HSB_PLAN_FP4,
    PLAN_DIGITS = HSB_PLAN_DIGITS,
    PLAN_INCREMENTAL = HSB_PLAN_INCREMENTAL
};

// Which plan runs (variant, this J, the precision option), or HSB_EUNSUPPORTED.
//   FP32:  the plain FP32 per-step plan, always.
//   MIXED: dSB with J exact in FP4 and N <= 2048 -> persistent FP4 plan;
//          otherwise the integer-digit plan (N <= 16384).
//   AUTO:  the FP4 plan where MIXED would take it; the digit plan for bSB and
//          for dSB with integer J in [-127, 127] (both as accurate as FP32 or
//          exact); FP32 otherwise.
int choose_plan(const hsb_ctx *h, int variant, int *plan) {
    const bool fp4_ok = h->j_fp4_exact && hsb::persistent_supported(h->N);
    const bool dig_ok = h->N <= hsb::i8_max_n();
    if (h->precision == HSB_PREC_FP32) {
        *plan = PLAN_FP32;
    } else if (h->precision == HSB_PREC_INCREMENTAL) {
        if (variant != HSB_DSB || !h->j_i8_exact || !dig_ok)
            return fail(HSB_EUNSUPPORTED, "INCREMENTAL precision needs dSB, integer J in "
                                          "[-127, 127] and N <= %d", hsb::i8_max_n());
        *plan = PLAN_INCREMENTAL;
    } else if (h->precision == HSB_PREC_DIGITS) {
        if (!dig_ok) return fail(HSB_EUNSUPPORTED, "DIGITS precision needs N <= %d", hsb::i8_max_n());
        *plan = PLAN_DIGITS;
    } else if (h->precision == HSB_PREC_MIXED) {
        if (fp4_ok)
            *plan = PLAN_FP4;
        else if (dig_ok)
            *plan = PLAN_DIGITS;
        else
            return fail(HSB_EUNSUPPORTED, "MIXED precision needs N <= %d", hsb::i8_max_n());
    } else {
        if (fp4_ok)
            *plan = PLAN_FP4;
        else if (dig_ok && (variant == HSB_BSB || h->j_i8_exact))
            *plan = PLAN_DIGITS;
        else
            *plan = PLAN_FP32;
    }
    return HSB_OK;
}

}  // namespace

extern "C" int hsb_plan_info(hsb_ctx *h, int variant, int *precision) {
    if (!h || !precision) return fail(HSB_EINVAL, "hsb_plan_info: NULL argument");
    if (variant != HSB_BSB && variant != HSB_DSB)
        return fail(HSB_EINVAL, "variant must be HSB_BSB (0) or HSB_DSB (1)");
    int plan = 0;
    const int rc = choose_plan(h, variant, &plan);
    if (rc == HSB_OK)
        *precision = plan == PLAN_FP32 ? HSB_PREC_FP32
                     : plan == PLAN_INCREMENTAL ? HSB_PREC_INCREMENTAL : HSB_PREC_MIXED;
    return rc;
}

namespace {

// Queue the device work of one run on s: state set-up, the plan's steps and
// the output.  Returns without waiting for it, except where the bSB digit
// plans check the start state.
int enqueue_run(hsb_ctx *h, const hsb_run_args *a, int &plan, hipStream_t s, int tile) {
    const int Ns = a->schedule_steps > 0 ? a->schedule_steps : a->start_step + a->steps;
    const int N = h->N, Npad = h->Npad, R = a->R;
    const int Rpad = round_up(R, hsb::kTile);
    int rc = HSB_OK;
    rc = ensure_state(h, Rpad);
    if (rc != HSB_OK) return rc;
    hsb::StateBufs &b = h->b;
    const float amp = (float)h->init_amp;
    const int interval = h->interval;

    // state set-up (eq. (16)-(22) start from x(t_0), y(t_0))
    if (a->x0)
        HIP_TRY(hsb::launch_load_state(b.X, b.Y, a->x0, a->y0, N, R, Npad, Rpad, s));
    else {
        HIP_TRY(hipMemcpyAsync(h->d_seed, h->h_seed, sizeof(uint64_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hsb::launch_init_seeded(b.X, b.Y, N, R, Npad, Rpad, Rpad, 0, amp, s, h->d_seed));
    }
    HIP_TRY(hsb::launch_fill_gamma(b.gamma, a->gamma_rep, a->gamma, R, Rpad, s));
    HIP_TRY(hsb::launch_reset_tracking(b, Rpad, s));
    // cancellation: the stop word of the per-step plans, polled after samples
    const int32_t *cancel = h->cancellable && h->cancel_opt ? h->d_cancel : nullptr;
    b.stop = h->d_stop;
    b.tstop = nullptr;
    HIP_TRY(hsb::launch_stop_init(b.stop, s));
    const bool nh = a->thermostat == HSB_THERMO_NOSE_HOOVER;
    if (nh) {
        if (h->nh_cap < Rpad) {
            // xi: two slots; partials: two sets of per-wave (32- or 64-row)
            // partials for the fused steps
            const size_t parts = 2 * (size_t)(Npad / 32);
            if (h->nh.xi) (void)hipFree(h->nh.xi);
            if (h->nh.part) (void)hipFree(h->nh.part);
            h->nh.xi = h->nh.part = nullptr;
            h->nh_cap = 0;
            HIP_TRY(hipMalloc((void **)&h->nh.xi, sizeof(double) * 2 * Rpad));
            HIP_TRY(hipMalloc((void **)&h->nh.part, sizeof(double) * parts * Rpad));
            h->nh_cap = Rpad;
        }
        // dt as the step kernels use it: a float
        h->nh.c = (double)a->dt * a->nh_inv_mass;
        h->nh.NT = (double)N * a->nh_temperature;
        HIP_TRY(hsb::launch_nh_init(h->nh, a->xi0, b.gamma, R, Rpad, s));
    }

    b.trace_e = a->trace_energy;
    b.trace_t = a->trace_tinst;
    b.trace_k0 = a->start_step;
    b.trace_interval = interval;
    h->timer.reset(h->timing != 0);
    const float a0 = a->a0, c0 = a->c0, dt = a->dt;
    const float a0dt = a0 * dt;
    const int k0 = a->start_step, k1 = a->start_step + a->steps;
    auto is_sample = [&](int m) { return m == k1 || (m > k0 && m % interval == 0); };
    auto sample = [&](int m) -> int {
        int nblk;
        if (h->j_int_exact) {
            HIP_TRY(hsb::launch_energy_fp32(h->dJ, b.X, b.epart, Npad, Rpad, s, b.stop));
            nblk = Npad / 32;
        } else {
            HIP_TRY(hsb::launch_energy_f64(h->dJ, b.X, b.epart, Npad, Rpad, s, b.stop));
            nblk = Npad / 64;
        }
        HIP_TRY(hsb::launch_best(b, nblk, N, R, Rpad, m, s));
        // a cancel request seen here stops the run at this sample point
        if (cancel && m < k1) HIP_TRY(hsb::launch_poll_cancel(cancel, b.stop, m, s));
        return HSB_OK;
    };

    if (a->variant == HSB_BSB && plan != PLAN_FP32 && (a->x0 || h->init_amp > 1.0)) {
        // the digit representations of x need |x| <= 1 in the start state (the
        // walls of eqs. (18)-(21) keep it so afterwards).  A seeded state with
        // amplitude <= 1 has it by construction: amp v with v in (-1, 1).
        if (!h->d_flag) HIP_TRY(hipMalloc((void **)&h->d_flag, sizeof(int32_t)));
        int32_t over = 0;
        HIP_TRY(hsb::launch_bound_check(b.X, (size_t)Npad * Rpad, h->d_flag, s));
        HIP_TRY(hipMemcpyAsync(&over, h->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (over) {
            if (h->precision != HSB_PREC_AUTO)
                return fail(HSB_EUNSUPPORTED,
                            "bSB on the FP4 or digit plan needs |x| <= 1 and finite in the "
                            "start state");
            plan = PLAN_FP32;
        }
    }
    if (plan == PLAN_DIGITS && !h->i8) {
        rc = hsb::i8_create(h->hJ.data(), N, &h->i8);
        if (rc != HSB_OK) return fail(rc, "%s", hsb::i8_error());
    }
    if (plan == PLAN_DIGITS) {
        hsb::I8Run ir{};
        ir.variant = a->variant;
        ir.N = N; ir.Nst = Npad; ir.Rpad = Rpad; ir.R = R;
        ir.k0 = k0; ir.k1 = k1; ir.Ns = Ns; ir.interval = interval;
        ir.a0 = a0; ir.c0 = c0; ir.dt = dt;
        ir.nh = nh ? &h->nh : nullptr;
        ir.tile = tile;
        ir.cancel = cancel;
        ir.local_exchange = h->local_exchange;
        rc = hsb::i8_run(h->i8, ir, b, h->dJ, s, h->timer);
        if (rc != HSB_OK) return fail(rc, "%s", hsb::i8_error());
    } else if (plan == PLAN_INCREMENTAL) {
        const size_t need = (size_t)Rpad * Npad;
        if (h->inc_cap < need) {
            if (h->inc.F) (void)hipFree(h->inc.F);
            if (h->inc.list) (void)hipFree(h->inc.list);
            if (h->inc.cnt) (void)hipFree(h->inc.cnt);
            h->inc = hsb::IncState{};
            h->inc_cap = 0;
            HIP_TRY(hipMalloc((void **)&h->inc.F, sizeof(int32_t) * need));
            HIP_TRY(hipMalloc((void **)&h->inc.list, sizeof(int32_t) * need));
            HIP_TRY(hipMalloc((void **)&h->inc.cnt, sizeof(int32_t) * 2 * Rpad));
            h->inc_cap = need;
        }
        HIP_TRY(hsb::launch_inc_init(h->dJ, b.X, h->inc, N, Npad, Rpad, R, s));
        if (a->steps == 0) {
            rc = sample(k0);
            if (rc) return rc;
        }
        size_t nrun = 0;
        for (int k = k0; k < k1; ++k) {
            const float ak = (a0 * (float)k) / (float)Ns;
            const float p = a0 - ak;
            HIP_TRY(h->timer.begin(s));
            HIP_TRY(hsb::launch_inc_step(h->dJ, b.X, b.Y, b.gamma, h->inc, k - k0, N, Npad, Rpad,
                                         R, p, c0, dt, a0dt, s, b.stop));
            ++nrun;
            if (is_sample(k + 1)) {
                HIP_TRY(h->timer.end(s, nrun));
                nrun = 0;
                rc = sample(k + 1);
                if (rc) return rc;
            }
        }
    } else if (plan == PLAN_FP4) {
        if (!h->pj) {
            rc = hsb::persistent_create(h->hJ.data(), N, &h->pj);
            if (rc != HSB_OK) return fail(rc, "%s", hsb::persistent_error());
        }
        hsb::PersistentRun pr{};
        pr.X = b.X; pr.Y = b.Y; pr.gamma = b.gamma;
        pr.Npad = Npad; pr.Rpad = Rpad; pr.R = R;
        pr.k0 = k0; pr.k1 = k1; pr.Ns = Ns; pr.interval = interval;
        pr.a0 = a0; pr.c0 = c0; pr.dt = dt;
        pr.epart = b.epart;
        pr.local_exchange = h->local_exchange;
        pr.tile = tile;
        pr.cancel = cancel;
        pr.nh = nh ? &h->nh : nullptr;
        rc = hsb::persistent_run(h->pj, a->variant, pr, b, N, s, h->timer);
        if (rc != HSB_OK) return fail(rc, "%s", hsb::persistent_error());
    } else {
        if (a->steps == 0) {
            rc = sample(k0);
            if (rc) return rc;
        } else {
            HIP_TRY(hsb::launch_make_operand(b.B[0], b.X, a->variant, Npad, Rpad, s));
            int cur = 0;
            size_t nrun = 0;  // step launches since the last energy sample
            for (int k = k0; k < k1; ++k) {
                // a(t_k) = a0 k / Ns in single precision; p = a0 - a(t_k)
                const float ak = (a0 * (float)k) / (float)Ns;
                const float p = a0 - ak;
                HIP_TRY(h->timer.begin(s));
                if (nh) {  // the thermostat fused into the step: slots alternate
                    const int j = k - k0, np = Npad / 32;
                    hsb::NHFused f;
                    f.xi_in = h->nh.xi + (size_t)(j & 1) * Rpad;
                    f.xi_out = h->nh.xi + (size_t)((j + 1) & 1) * Rpad;
                    f.part_out = h->nh.part + (size_t)(j & 1) * np * Rpad;
                    f.part_in = h->nh.part + (size_t)((j + 1) & 1) * np * Rpad;
                    f.nparts = np;
                    f.first = j == 0;
                    f.c = h->nh.c;
                    f.NT = h->nh.NT;
                    HIP_TRY(hsb::launch_step_fp32(a->variant, h->dJ, b.B[cur], b.B[cur ^ 1], b.X,
                                                  b.Y, b.gamma, Npad, Rpad, p, c0, dt, a0dt, s, &f,
                                                  b.stop));
                } else {
                    HIP_TRY(hsb::launch_step_fp32(a->variant, h->dJ, b.B[cur], b.B[cur ^ 1], b.X,
                                                  b.Y, b.gamma, Npad, Rpad, p, c0, dt, a0dt, s,
                                                  nullptr, b.stop));
                }
                ++nrun;
                cur ^= 1;
                if (is_sample(k + 1)) {
                    HIP_TRY(h->timer.end(s, nrun));
                    nrun = 0;
                    rc = sample(k + 1);
                    if (rc) return rc;
                }
            }
            if (nh)  // xi after the last step, from its slot and partials, into slot 0
                HIP_TRY(hsb::launch_nh_final(h->nh.xi, h->nh.part, Npad / 32, R, Rpad, h->nh.xi,
                                             h->nh.c, h->nh.NT, k1 - k0, k0, b.stop, s));
        }
    }
    HIP_TRY(hsb::launch_output(b, N, R, Rpad, h->return_best, a->spins, a->energy, a->x_out,
                               a->y_out, a->best_energy, a->final_energy, a->best_step, s));
    HIP_TRY(hsb::launch_output_stop(b.stop, b.tstop, R, k1, a->stop_step, b.status, s));
    if (nh && a->xi_out) HIP_TRY(hsb::launch_copy_f64(a->xi_out, h->nh.xi, R, s));
    // status: bit 0 a non-finite state, bit 1 an exchange wait of the
    // persistent kernels that timed out
    return HSB_OK;
}

// Everything the device work queued by enqueue_run depends on: the arguments,
// the options, the plan, and the buffers it uses (by address and generation).
std::vector<uint64_t> run_key(const hsb_ctx *h, const hsb_run_args *a, int plan, int tile) {
    auto fb = [](float v) {
        uint32_t u;
        std::memcpy(&u, &v, sizeof u);
        return (uint64_t)u;
    };
    auto pb = [](const void *q) { return (uint64_t)(uintptr_t)q; };
    auto db = [](double v) {
        uint64_t u;
        std::memcpy(&u, &v, sizeof u);
        return u;
    };
    uint64_t amp;
    std::memcpy(&amp, &h->init_amp, sizeof amp);
    // (not the seed: the queued work reads it from the context's pinned slot)
    return {(uint64_t)a->variant, (uint64_t)a->steps, (uint64_t)a->R, (uint64_t)a->start_step,
            (uint64_t)a->schedule_steps, fb(a->a0), fb(a->c0), fb(a->dt), fb(a->gamma),
            pb(a->gamma_rep), pb(a->x0), pb(a->y0), pb(a->x_out), pb(a->y_out), pb(a->spins),
            pb(a->energy), pb(a->best_energy), pb(a->final_energy), pb(a->best_step),
            pb(a->trace_energy), pb(a->trace_tinst), pb(a->stop_step), (uint64_t)a->thermostat,
            db(a->nh_inv_mass),
            db(a->nh_temperature), pb(a->xi0), pb(a->xi_out), amp,
            (uint64_t)h->interval, (uint64_t)h->return_best, (uint64_t)h->local_exchange,
            (uint64_t)h->cancel_opt,
            (uint64_t)plan, pb(h->b.X), (uint64_t)h->Rpad_cap, h->state_gen, pb(h->pj),
            h->pj ? hsb::persistent_gen(h->pj) : 0, (uint64_t)tile};
}

// Launch the cached graph on the context's stream, ordered after the work
// already queued on s and before whatever s gets next.
int graph_launch(hsb_ctx *h, hipStream_t s) {
    HIP_TRY(hipEventRecord(h->gev_in, s));
    HIP_TRY(hipStreamWaitEvent(h->gstream, h->gev_in, 0));
    HIP_TRY(hipGraphLaunch(h->gexec, h->gstream));
    HIP_TRY(hipEventRecord(h->gev_out, h->gstream));
    HIP_TRY(hipStreamWaitEvent(s, h->gev_out, 0));
    ++h->glaunches;
    return HSB_OK;
}

// A run through the graph cache: the first call with a key runs eagerly
// (allocating what the run needs); the next call with the same key captures
// the same queued work on the context's stream into a graph and launches it;
// later calls with that key launch the graph again.  Any other key, or a
// buffer reallocated in between (a new generation), drops the graph.
int run_graph(hsb_ctx *h, const hsb_run_args *a, int &plan, hipStream_t s, int tile) {
    const std::vector<uint64_t> key = run_key(h, a, plan, tile);
    if (h->gexec && key == h->gkey) return graph_launch(h, s);
    if (h->gseen && key == h->gkey) {
        if (!h->gstream) {
            HIP_TRY(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&h->gev_in, hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&h->gev_out, hipEventDisableTiming));
        }
        HIP_TRY(hipEventRecord(h->gev_in, s));
        HIP_TRY(hipStreamWaitEvent(h->gstream, h->gev_in, 0));
        HIP_TRY(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_run(h, a, plan, h->gstream, tile);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(h->gstream, &g);
        if (rc == HSB_OK && e != hipSuccess) rc = hip_fail(e, "capturing the run");
        // the captured work must be that of the key: nothing reallocated
        if (rc == HSB_OK && run_key(h, a, plan, tile) != key)
            rc = fail(HSB_EDEVICE, "run buffers changed while capturing");
        if (rc == HSB_OK) {
            const hipError_t ei = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
            if (ei != hipSuccess) {
                h->gexec = nullptr;
                rc = hip_fail(ei, "instantiating the run graph");
            }
        }
        if (g) (void)hipGraphDestroy(g);
        if (rc != HSB_OK) {
            // nothing of a failed capture ran: queue the run eagerly instead
            graph_drop(h);
            (void)hipGetLastError();
            return enqueue_run(h, a, plan, s, tile);
        }
        return graph_launch(h, s);
    }
    graph_drop(h);
    const int rc = enqueue_run(h, a, plan, s, tile);
    if (rc != HSB_OK) return rc;
    h->gkey = run_key(h, a, plan, tile);  // after the run: the buffers it grew are part of it
    h->gseen = true;
    return HSB_OK;
}

// Result-invariant kernel variants of a plan (the autotuner's candidates).
int tile_count(int plan, int variant, int thermostat) {
    if (plan == PLAN_FP4) return thermostat == HSB_THERMO_NOSE_HOOVER ? 1 : hsb::persistent_tiles(variant);
    if (plan == PLAN_DIGITS) return hsb::i8_tiles();
    return 1;
}

// Device staging of R replicas' spins and energies (hsb_run's outputs, and
// the tuner's throw-away outputs).
int ensure_staging(hsb_ctx *h, int R) {
    const size_t need = (size_t)R * h->N;
    if (need <= h->run_cap && h->d_energy) return HSB_OK;  // N is fixed: R fits too
    if (h->d_spins) (void)hipFree(h->d_spins);
    if (h->d_energy) (void)hipFree(h->d_energy);
    h->d_spins = nullptr;
    h->d_energy = nullptr;
    h->run_cap = 0;
    HIP_TRY(hipMalloc((void **)&h->d_spins, need));
    HIP_TRY(hipMalloc((void **)&h->d_energy, sizeof(double) * (size_t)R));
    h->run_cap = need;
    return HSB_OK;
}

// The kernel variant of a run: the forced option; else, with AUTOTUNE on, the
// tuned choice for this plan and shape (timed now on a short run of the same
// shape if the cache has none); else the default 0.
int choose_tile(hsb_ctx *h, const hsb_run_args *a, int plan, hipStream_t s, int *tile) {
    const int n = tile_count(plan, a->variant, a->thermostat);
    *tile = 0;
    if (h->tile >= 0) {
        if (h->tile >= n)
            return fail(HSB_EINVAL, "TILE = %d, but this plan has %d kernel variants", h->tile, n);
        *tile = h->tile;
        return HSB_OK;
    }
    if (!h->autotune || n <= 1 || a->steps == 0) return HSB_OK;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap));
    static const char *plan_name[] = {"fp32", "fp4", "digits", "incremental"};
    const int Npad = plan == PLAN_FP4 ? (h->N + 255) / 256 * 256
                                      : (h->N + hsb::kI8SpinTile - 1) / hsb::kI8SpinTile * hsb::kI8SpinTile;
    char key[160];
    std::snprintf(key, sizeof key, "gfx950/%s/%s/N%d/R%d/J%s/T%d", plan_name[plan],
                  a->variant == HSB_BSB ? "bsb" : "dsb", Npad, round_up(a->R, hsb::kTile),
                  h->j_i8_exact ? "int8" : "real", a->thermostat);
    int c = 0;
    if (hsb::tune_lookup(key, &c) && c < n) {
        *tile = c;
        return HSB_OK;
    }
    if (cap != hipStreamCaptureStatusNone) return HSB_OK;  // no timing inside a capture
    // time every variant on the first steps of this run's schedule (outputs
    // to the context's staging, nothing of the caller's written)
    int rc = ensure_staging(h, a->R);
    if (rc != HSB_OK) return rc;
    hsb_run_args t = *a;
    t.steps = std::min(a->steps, 200);
    t.schedule_steps = a->schedule_steps > 0 ? a->schedule_steps : a->start_step + a->steps;
    t.spins = h->d_spins;
    t.energy = h->d_energy;
    t.x_out = t.y_out = nullptr;
    t.best_energy = t.final_energy = nullptr;
    t.best_step = nullptr;
    t.trace_energy = t.trace_tinst = nullptr;
    t.xi_out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "tuner events");
    }
    const int timing = h->timing;
    h->timing = 0;
    std::vector<double> ms(n, 0.0);
    for (int v = 0; v < n && rc == HSB_OK; ++v) {
        for (int rep = 0; rep < 2 && rc == HSB_OK; ++rep) {  // the first warms up
            int p = plan;
            he = hipEventRecord(e0, s);
            if (he == hipSuccess) rc = enqueue_run(h, &t, p, s, v);
            if (rc == HSB_OK && he == hipSuccess) he = hipEventRecord(e1, s);
            if (rc == HSB_OK && he == hipSuccess) he = hipEventSynchronize(e1);
            float f = 0.0f;
            if (rc == HSB_OK && he == hipSuccess) he = hipEventElapsedTime(&f, e0, e1);
            if (rc == HSB_OK && he != hipSuccess) rc = hip_fail(he, "timing a kernel variant");
            ms[v] = f;
        }
    }
    h->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != HSB_OK) return rc;
    *tile = (int)(std::min_element(ms.begin(), ms.end()) - ms.begin());
    (void)hsb::tune_store(key, *tile, ms);  // unwritable cache: tuned again next process
    return HSB_OK;
}

// Everything a queued batch's device work depends on: the team table (the
// instances' J stores, the outputs, seeds and parameters), the shared run
// arguments and the generation of the lead context's queue buffers.
std::vector<uint64_t> batch_key(const hsb_ctx *lead, const std::vector<hsb::QTeam> &qt,
                                const hsb::QRun &qr) {
    static_assert(sizeof(hsb::QTeam) % 8 == 0, "team records are whole words");
    std::vector<uint64_t> k(qt.size() * sizeof(hsb::QTeam) / 8 + 8);
    if (!qt.empty()) std::memcpy(k.data(), qt.data(), qt.size() * sizeof(hsb::QTeam));
    uint64_t *t = k.data() + qt.size() * sizeof(hsb::QTeam) / 8;
    uint32_t f[3];
    std::memcpy(&f[0], &qr.a0, 4);
    std::memcpy(&f[1], &qr.dt, 4);
    std::memcpy(&f[2], &qr.amp, 4);
    t[0] = (uint64_t)(uint32_t)qr.steps;
    t[1] = (uint64_t)(uint32_t)qr.interval;
    t[2] = (uint64_t)qr.return_best | ((uint64_t)qr.local_exchange << 8);
    t[3] = f[0];
    t[4] = f[1];
    t[5] = f[2];
    t[6] = lead->qwork ? hsb::queue_gen(lead->qwork) : 0;
    t[7] = (uint64_t)qt.size();
    return k;
}

int ensure_graph_stream(hsb_ctx *h) {
    if (!h->gstream) {
        HIP_TRY(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&h->gev_in, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&h->gev_out, hipEventDisableTiming));
    }
    return HSB_OK;
}

// A queued batch through the lead context's graph cache: the first call with a
// key runs eagerly (allocating and uploading what it needs), the next call
// with that key captures the same work on the context's stream and launches
// it, later calls launch it again; any other key drops the graph.
int batch_graph(hsb_ctx *lead, const std::vector<hsb::QTeam> &qt, const hsb::QRun &qr,
                hipStream_t s, int policy) {
    std::vector<uint64_t> key = batch_key(lead, qt, qr);
    key.push_back((uint64_t)policy);
    auto launch = [&]() -> int {
        HIP_TRY(hipEventRecord(lead->gev_in, s));
        HIP_TRY(hipStreamWaitEvent(lead->gstream, lead->gev_in, 0));
        HIP_TRY(hipGraphLaunch(lead->bgexec, lead->gstream));
        HIP_TRY(hipEventRecord(lead->gev_out, lead->gstream));
        HIP_TRY(hipStreamWaitEvent(s, lead->gev_out, 0));
        ++lead->glaunches;
        return HSB_OK;
    };
    if (lead->bgexec && key == lead->bgkey) return launch();
    if (lead->bgseen && key == lead->bgkey) {
        int rc = ensure_graph_stream(lead);
        if (rc != HSB_OK) return rc;
        HIP_TRY(hipEventRecord(lead->gev_in, s));
        HIP_TRY(hipStreamWaitEvent(lead->gstream, lead->gev_in, 0));
        HIP_TRY(hipStreamBeginCapture(lead->gstream, hipStreamCaptureModeThreadLocal));
        hsb::KernelTimer off;
        rc = hsb::queue_run(lead->qwork, qt, qr, policy, lead->gstream, off);
        if (rc != HSB_OK) (void)fail(rc, "%s", hsb::queue_error());
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(lead->gstream, &g);
        if (rc == HSB_OK && e != hipSuccess) rc = hip_fail(e, "capturing the batch");
        std::vector<uint64_t> key_after = batch_key(lead, qt, qr);
        key_after.push_back((uint64_t)policy);
        if (rc == HSB_OK && key_after != key)
            rc = fail(HSB_EDEVICE, "batch buffers changed while capturing");
        if (rc == HSB_OK) {
            const hipError_t ei = hipGraphInstantiate(&lead->bgexec, g, nullptr, nullptr, 0);
            if (ei != hipSuccess) {
                lead->bgexec = nullptr;
                rc = hip_fail(ei, "instantiating the batch graph");
            }
        }
        if (g) (void)hipGraphDestroy(g);
        if (rc != HSB_OK) {  // nothing of a failed capture ran: queue it eagerly
            batch_graph_drop(lead);
            (void)hipGetLastError();
            const int r2 = hsb::queue_run(lead->qwork, qt, qr, policy, s, lead->timer);
            return r2 == HSB_OK ? HSB_OK : fail(r2, "%s", hsb::queue_error());
        }
        return launch();
    }
    batch_graph_drop(lead);
    const int rc = hsb::queue_run(lead->qwork, qt, qr, policy, s, lead->timer);
    if (rc != HSB_OK) return fail(rc, "%s", hsb::queue_error());
    lead->bgkey = batch_key(lead, qt, qr);  // after the run: what it grew is part of it
    lead->bgkey.push_back((uint64_t)policy);
    lead->bgseen = true;
    return HSB_OK;
}

}  // namespace

namespace {

// The argument checks shared by the run entry points (all on the
// host, before any device work).
int check_run_args(const hsb_run_args *a) {
    if (a->variant != HSB_BSB && a->variant != HSB_DSB)
        return fail(HSB_EINVAL, "variant must be HSB_BSB (0) or HSB_DSB (1)");
    if (a->steps < 0) return fail(HSB_EINVAL, "steps must be >= 0");
    if (a->R < 1 || a->R > (1 << 22)) return fail(HSB_EINVAL, "R must be in [1, 4194304]");
    if (a->start_step < 0) return fail(HSB_EINVAL, "start_step must be >= 0");
    if ((long long)a->start_step + a->steps > 2147483647LL)
        return fail(HSB_EINVAL, "start_step + steps overflows");
    const int Ns = a->schedule_steps > 0 ? a->schedule_steps : a->start_step + a->steps;
    if (a->schedule_steps < 0 || Ns < a->start_step + a->steps)
        return fail(HSB_EINVAL, "schedule_steps must be 0 or >= start_step + steps");
    if (!(std::isfinite(a->a0) && std::isfinite(a->c0) && std::isfinite(a->dt) &&
          std::isfinite(a->gamma)))
        return fail(HSB_EINVAL, "a0, c0, dt and gamma must be finite");
    if (!(a->dt > 0.0f)) return fail(HSB_EINVAL, "dt must be > 0");
    if (!(a->gamma >= 0.0f)) return fail(HSB_EINVAL, "gamma must be >= 0");
    if (!a->spins || !a->energy) return fail(HSB_EINVAL, "spins and energy are required");
    if ((a->x0 == nullptr) != (a->y0 == nullptr))
        return fail(HSB_EINVAL, "x0 and y0 must be given together");
    if (a->thermostat != HSB_THERMO_HEAT && a->thermostat != HSB_THERMO_NOSE_HOOVER)
        return fail(HSB_EINVAL, "thermostat must be HSB_THERMO_HEAT (0) or HSB_THERMO_NOSE_HOOVER (1)");
    if (a->thermostat == HSB_THERMO_NOSE_HOOVER) {
        if (!(std::isfinite(a->nh_inv_mass) && a->nh_inv_mass >= 0.0 &&
              std::isfinite(a->nh_temperature) && a->nh_temperature >= 0.0))
            return fail(HSB_EINVAL, "nh_inv_mass and nh_temperature must be finite and >= 0");
    } else if (a->nh_inv_mass != 0.0 || a->nh_temperature != 0.0 || a->xi0 || a->xi_out) {
        return fail(HSB_EINVAL, "nh_inv_mass, nh_temperature, xi0 and xi_out need "
                                "HSB_THERMO_NOSE_HOOVER");
    }
    return HSB_OK;
}

}  // namespace

extern "C" int hsb_run_ex(hsb_ctx *h, const hsb_run_args *a) {
    g_err[0] = 0;
    if (!h || !a) return fail(HSB_EINVAL, "hsb_run_ex: NULL argument");
    if (a->struct_size != sizeof(hsb_run_args))
        return fail(HSB_EINVAL, "hsb_run_ex: struct_size %zu != %zu", a->struct_size,
                    sizeof(hsb_run_args));
    {
        const int rc = check_run_args(a);
        if (rc != HSB_OK) return rc;
    }
    int plan = 0;
    int rc = choose_plan(h, a->variant, &plan);
    if (rc != HSB_OK) return rc;
    // the persistent bSB kernel's thermostat variant takes no cancel requests:
    // in a cancellable context the digit plan runs it
    if (a->thermostat == HSB_THERMO_NOSE_HOOVER && plan == PLAN_FP4 && a->variant == HSB_BSB &&
        h->cancellable && h->cancel_opt)
        plan = h->N <= hsb::i8_max_n() ? PLAN_DIGITS : PLAN_FP32;
    if (a->thermostat == HSB_THERMO_NOSE_HOOVER && plan == PLAN_INCREMENTAL)
        return fail(HSB_EUNSUPPORTED, "the thermostat does not run on the INCREMENTAL plan");
    HIP_TRY(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)a->stream;
    const int R = a->R;
    if (!h->d_seed) {
        HIP_TRY(hipMalloc((void **)&h->d_seed, sizeof(uint64_t)));
        HIP_TRY(hipHostMalloc((void **)&h->h_seed, sizeof(uint64_t), hipHostMallocDefault));
    }
    // no queued work of an earlier call reads the slot any more: every call
    // ends by synchronising its stream
    *h->h_seed = a->seed;
    if (a->gamma_rep) {
        std::vector<float> g(R);
        HIP_TRY(hipMemcpyAsync(g.data(), a->gamma_rep, sizeof(float) * R, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int r = 0; r < R; ++r)
            if (!(std::isfinite(g[r]) && g[r] >= 0.0f))
                return fail(HSB_EINVAL, "gamma_rep[%d] = %g must be finite and >= 0", r, g[r]);
    }
    // graphs for the persistent FP4 runs (their queued work is free of host
    // round trips once the run's buffers exist; for bSB, when no start-state
    // check is needed), unless the caller is capturing the stream itself
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap));
    const bool graphable = h->graph && plan == PLAN_FP4 && !h->timing &&
                           cap == hipStreamCaptureStatusNone &&
                           (a->variant == HSB_DSB || (!a->x0 && h->init_amp <= 1.0));
    int tile = 0;
    rc = choose_tile(h, a, plan, s, &tile);
    if (rc != HSB_OK) return rc;
    rc = graphable ? run_graph(h, a, plan, s, tile) : enqueue_run(h, a, plan, s, tile);
    if (rc != HSB_OK) return rc;
    // status: bit 0 a non-finite state, bit 1 an exchange wait of the
    // persistent kernels that timed out
    int32_t status = 0;
    HIP_TRY(hipMemcpyAsync(&status, h->b.status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // a cancel request is used up by the run in progress, seen or not
    __atomic_store_n(h->h_cancel, 0, __ATOMIC_SEQ_CST);
    if (status & 2) return fail(HSB_EDEVICE, "FP4 persistent kernel: exchange wait timed out");
    h->last_plan = plan;
    h->last_tile = tile;
    if (status & 4) return fail(HSB_ECANCELED, "the run was cancelled at a sample point");
    if (status & 1) return fail(HSB_ENUMERIC, "a replica's state became non-finite");
    return HSB_OK;
}

extern "C" int hsb_run(hsb_ctx *h, int variant, float a0, float c0, float dt, float gamma,
                       int steps, int R, uint64_t seed, int8_t *spins, double *energy) {
    g_err[0] = 0;
    if (!h) return fail(HSB_EINVAL, "hsb_run: NULL context");
    if (!spins || !energy) return fail(HSB_EINVAL, "hsb_run: spins and energy are required");
    if (R < 1 || R > (1 << 22)) return fail(HSB_EINVAL, "R must be in [1, 4194304]");
    HIP_TRY(hipSetDevice(h->device));
    const size_t need = (size_t)R * h->N;
    {
        const int rc = ensure_staging(h, R);
        if (rc != HSB_OK) return rc;
    }
    hsb_run_args a;
    std::memset(&a, 0, sizeof(a));
    a.struct_size = sizeof(a);
    a.variant = variant;
    a.steps = steps;
    a.R = R;
    a.a0 = a0;
    a.c0 = c0;
    a.dt = dt;
    a.gamma = gamma;
    a.seed = seed;
    a.spins = h->d_spins;
    a.energy = h->d_energy;
    a.stream = h->stream;
    const int rc = hsb_run_ex(h, &a);
    if (rc != HSB_OK && rc != HSB_ENUMERIC && rc != HSB_ECANCELED) return rc;
    HIP_TRY(hipMemcpyAsync(spins, h->d_spins, need, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(energy, h->d_energy, sizeof(double) * R, hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return rc;
}

extern "C" int hsb_run_ex_noalloc(hsb_ctx *h, const hsb_run_args *a) {
    g_err[0] = 0;
    if (!h || !a) return fail(HSB_EINVAL, "hsb_run_ex_noalloc: NULL argument");
    if (a->struct_size != sizeof(hsb_run_args))
        return fail(HSB_EINVAL, "hsb_run_ex_noalloc: struct_size %zu != %zu", a->struct_size,
                    sizeof(hsb_run_args));
    int rc = check_run_args(a);
    if (rc != HSB_OK) return rc;
    if (a->variant != HSB_DSB)
        return fail(HSB_EUNSUPPORTED, "hsb_run_ex_noalloc runs dSB only");
    if (a->thermostat != HSB_THERMO_HEAT || a->trace_energy || a->trace_tinst)
        return fail(HSB_EUNSUPPORTED, "hsb_run_ex_noalloc runs neither the thermostat nor traces");
    int plan = 0;
    rc = choose_plan(h, HSB_DSB, &plan);
    if (rc != HSB_OK) return rc;
    if (plan != PLAN_FP4 || !h->pj)
        return fail(HSB_EUNSUPPORTED, "hsb_run_ex_noalloc needs the FP4 plan (J exact in FP4, "
                                      "N <= %d, precision AUTO or MIXED)",
                    hsb::persistent_max_n());
    HIP_TRY(hipSetDevice(h->device));
    void *base = nullptr;
    rc = scratch_address(h->device, &base);
    if (rc != HSB_OK) return rc;
    const int N = h->N, Npad = h->Npad, R = a->R;
    const int Rpad = round_up(R, hsb::kTile);
    // the state of the run, carved from the front of the scratch
    uint8_t *const s0 = static_cast<uint8_t *>(base);
    size_t used = 0;
    auto take = [&](size_t bytes) {
        used = (used + 255) / 256 * 256;
        void *p = s0 + used;
        used += bytes;
        return p;
    };
    const size_t nr = (size_t)Rpad, ns = (size_t)Npad * nr;
    hsb::StateBufs b{};
    b.X = static_cast<float *>(take(ns * sizeof(float)));
    b.Y = static_cast<float *>(take(ns * sizeof(float)));
    b.gamma = static_cast<float *>(take(nr * sizeof(float)));
    b.best_e = static_cast<double *>(take(nr * sizeof(double)));
    b.last_e = static_cast<double *>(take(nr * sizeof(double)));
    b.best_step = static_cast<int32_t *>(take(nr * sizeof(int32_t)));
    b.bad = static_cast<int32_t *>(take(nr * sizeof(int32_t)));
    b.best_s = static_cast<int8_t *>(take(ns));
    b.status = static_cast<int32_t *>(take(sizeof(int32_t)));
    int32_t *flag = static_cast<int32_t *>(take(sizeof(int32_t)));
    used = (used + 255) / 256 * 256;
    if (used >= HSB_NOALLOC_SCRATCH_BYTES)
        return fail(HSB_EINVAL, "hsb_run_ex_noalloc: R = %d at N = %d needs %zu bytes of state, "
                                "more than the %zu-byte scratch", R, N, used,
                    (size_t)HSB_NOALLOC_SCRATCH_BYTES);
    hipStream_t s = (hipStream_t)a->stream;
    if (a->gamma_rep) {  // checked on the device: no host copy of the array
        int32_t bad = 0;
        hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(1), 0, s, flag);
        hipLaunchKernelGGL(k_flag_bad_gamma, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s,
                           a->gamma_rep, R, flag);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (bad) return fail(HSB_EINVAL, "gamma_rep must be finite and >= 0");
    }
    const float amp = (float)h->init_amp;
    if (a->x0)
        HIP_TRY(hsb::launch_load_state(b.X, b.Y, a->x0, a->y0, N, R, Npad, Rpad, s));
    else
        HIP_TRY(hsb::launch_init_seeded(b.X, b.Y, N, R, Npad, Rpad, Rpad, a->seed, amp, s));
    HIP_TRY(hsb::launch_fill_gamma(b.gamma, a->gamma_rep, a->gamma, R, Rpad, s));
    HIP_TRY(hsb::launch_reset_tracking(b, Rpad, s));
    hsb::PersistentRun pr{};
    pr.X = b.X; pr.Y = b.Y; pr.gamma = b.gamma;
    pr.Npad = Npad; pr.Rpad = Rpad; pr.R = R;
    pr.k0 = a->start_step; pr.k1 = a->start_step + a->steps;
    pr.Ns = a->schedule_steps > 0 ? a->schedule_steps : a->start_step + a->steps;
    pr.interval = h->interval;
    pr.a0 = a->a0; pr.c0 = a->c0; pr.dt = a->dt;
    pr.local_exchange = h->local_exchange;
    pr.cancel = h->cancellable && h->cancel_opt ? h->d_cancel : nullptr;
    rc = hsb::persistent_run_in(s0 + used, HSB_NOALLOC_SCRATCH_BYTES - used, h->pj, pr, b, N, s);
    if (rc != HSB_OK) return fail(rc, "hsb_run_ex_noalloc: %s", hsb::persistent_error());
    HIP_TRY(hsb::launch_output(b, N, R, Rpad, h->return_best, a->spins, a->energy, a->x_out,
                               a->y_out, a->best_energy, a->final_energy, a->best_step, s));
    HIP_TRY(hsb::launch_output_stop(nullptr, b.tstop, R, pr.k1, a->stop_step, b.status, s));
    int32_t status = 0;
    HIP_TRY(hipMemcpyAsync(&status, b.status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    __atomic_store_n(h->h_cancel, 0, __ATOMIC_SEQ_CST);
    if (status & 2) return fail(HSB_EDEVICE, "FP4 persistent kernel: exchange wait timed out");
    h->last_plan = PLAN_FP4;
    if (status & 4) return fail(HSB_ECANCELED, "the run was cancelled at a sample point");
    if (status & 1) return fail(HSB_ENUMERIC, "a replica's state became non-finite");
    return HSB_OK;
}

extern "C" int hsb_run_batch(hsb_ctx *const *hs, int n_inst, const hsb_job *jobs, int n_jobs,
                             const hsb_batch_args *a) {
    g_err[0] = 0;
    if (!hs || !a || (n_jobs > 0 && !jobs)) return fail(HSB_EINVAL, "hsb_run_batch: NULL argument");
    if (a->struct_size != sizeof(hsb_batch_args))
        return fail(HSB_EINVAL, "hsb_run_batch: struct_size %zu != %zu", a->struct_size,
                    sizeof(hsb_batch_args));
    if (n_inst < 1 || n_jobs < 0) return fail(HSB_EINVAL, "n_inst must be >= 1, n_jobs >= 0");
    if (a->variant != HSB_BSB && a->variant != HSB_DSB)
        return fail(HSB_EINVAL, "variant must be HSB_BSB (0) or HSB_DSB (1)");
    if (a->steps < 0) return fail(HSB_EINVAL, "steps must be >= 0");
    if (!(std::isfinite(a->a0) && std::isfinite(a->dt) && a->dt > 0.0f))
        return fail(HSB_EINVAL, "a0 must be finite and dt finite and > 0");
    const double amp = a->init_amp == 0.0 ? 0.1 : a->init_amp;
    if (!(std::isfinite(amp) && amp > 0.0 && amp <= 1.0e6))
        return fail(HSB_EINVAL, "init_amp must be finite and > 0");
    const int interval = a->energy_interval == 0 ? 100 : a->energy_interval;
    if (interval < 1) return fail(HSB_EINVAL, "energy_interval must be >= 1");
    if (a->return_best != 0 && a->return_best != 1)
        return fail(HSB_EINVAL, "return_best must be 0 or 1");
    if (a->scheduler != HSB_SCHED_QUEUE && a->scheduler != HSB_SCHED_CLASSES)
        return fail(HSB_EINVAL, "scheduler must be HSB_SCHED_QUEUE (0) or HSB_SCHED_CLASSES (1)");
    for (int i = 0; i < n_inst; ++i) {
        if (!hs[i]) return fail(HSB_EINVAL, "hs[%d] is NULL", i);
        if (hs[i]->device != hs[0]->device)
            return fail(HSB_EINVAL, "all contexts must be on one device");
    }
    // plan of every job (the instance's precision option), FP4 jobs grouped by padded size
    std::map<int, std::vector<int>> classes;  // K blocks of 64 -> jobs
    std::vector<int> singles, queued;
    for (int j = 0; j < n_jobs; ++j) {
        const hsb_job &jb = jobs[j];
        if (jb.instance < 0 || jb.instance >= n_inst)
            return fail(HSB_EINVAL, "job %d: instance %d out of range", j, jb.instance);
        if (jb.R < 1 || jb.R > (1 << 22)) return fail(HSB_EINVAL, "job %d: R out of range", j);
        if (!std::isfinite(jb.c0)) return fail(HSB_EINVAL, "job %d: c0 must be finite", j);
        if (!(std::isfinite(jb.gamma) && jb.gamma >= 0.0f))
            return fail(HSB_EINVAL, "job %d: gamma must be finite and >= 0", j);
        if (!jb.spins || !jb.energy) return fail(HSB_EINVAL, "job %d: spins and energy required", j);
        int plan = 0;
        const int rc = choose_plan(hs[jb.instance], a->variant, &plan);
        if (rc != HSB_OK) return rc;
        // bSB's digit representation of x needs |x| <= 1 at the start
        if (plan == PLAN_FP4 && a->variant == HSB_DSB && a->scheduler == HSB_SCHED_QUEUE)
            queued.push_back(j);
        else if (plan == PLAN_FP4 && !(a->variant == HSB_BSB && amp > 1.0))
            classes[(hs[jb.instance]->N + 255) / 256 * 4].push_back(j);
        else
            singles.push_back(j);
    }
    hsb_ctx *lead = hs[0];
    HIP_TRY(hipSetDevice(lead->device));
    hipStream_t s = (hipStream_t)a->stream;
    int any_bad = 0;

    // jobs outside the FP4 plan: one run each (their contexts' own plans)
    for (int j : singles) {
        const hsb_job &jb = jobs[j];
        hsb_ctx *h = hs[jb.instance];
        const double amp0 = h->init_amp;
        const int int0 = h->interval, rb0 = h->return_best, tim0 = h->timing;
        h->init_amp = amp;
        h->interval = interval;
        h->return_best = a->return_best;
        h->timing = 0;
        h->cancellable = false;  // batches are not cancelled
        hsb_run_args ra;
        std::memset(&ra, 0, sizeof(ra));
        ra.struct_size = sizeof(ra);
        ra.variant = a->variant;
        ra.steps = a->steps;
        ra.R = jb.R;
        ra.a0 = a->a0;
        ra.c0 = jb.c0;
        ra.dt = a->dt;
        ra.gamma = jb.gamma;
        ra.seed = jb.seed;
        ra.spins = jb.spins;
        ra.energy = jb.energy;
        ra.stream = a->stream;
        const int rc = hsb_run_ex(h, &ra);
        h->cancellable = true;
        h->init_amp = amp0;
        h->interval = int0;
        h->return_best = rb0;
        h->timing = tim0;
        if (rc == HSB_ENUMERIC)
            any_bad = 1;
        else if (rc != HSB_OK)
            return rc;
    }

    // FP4 jobs; the lead context's timer (TIMING on) records their launches
    lead->timer.reset(lead->timing != 0);
    // dSB: every job in one persistent launch fed by the job queues
    if (!queued.empty()) {
        std::vector<hsb::QTeam> qt;
        for (int j : queued) {
            const hsb_job &jb = jobs[j];
            hsb_ctx *h = hs[jb.instance];
            if (!h->pj) {
                const int rc = hsb::persistent_create(h->hJ.data(), h->N, &h->pj);
                if (rc != HSB_OK) return fail(rc, "%s", hsb::persistent_error());
            }
            const int nkb = hsb::persistent_nkb(h->pj);
            for (int t0 = 0; t0 < jb.R; t0 += 32)
                qt.push_back(hsb::QTeam{hsb::persistent_jpk(h->pj), jb.spins, jb.energy, jb.seed,
                                        h->N, nkb, t0, std::min(32, jb.R - t0), jb.c0, jb.gamma});
        }
        if (!lead->qwork) {
            const int rc = hsb::queue_work_create(&lead->qwork);
            if (rc != HSB_OK) return fail(rc, "%s", hsb::queue_error());
        }
        hsb::QRun qr{};
        qr.steps = a->steps;
        qr.interval = interval;
        qr.return_best = a->return_best;
        qr.a0 = a->a0;
        qr.dt = a->dt;
        qr.amp = (float)amp;
        qr.local_exchange = lead->local_exchange;
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(s, &cap));
        // the queue placement policy: forced (TILE of the lead context), tuned
        // (AUTOTUNE), or longest-first
        int policy = 0;
        if (lead->tile >= 0) {
            if (lead->tile >= 2) return fail(HSB_EINVAL, "TILE = %d, but batch queues have 2 "
                                                         "placement policies", lead->tile);
            policy = lead->tile;
        } else if (lead->autotune && a->steps > 0) {
            long long wg = 0;
            for (const hsb::QTeam &q : qt) wg += q.nkb / 2;
            char key[160];
            std::snprintf(key, sizeof key, "gfx950/queue/dsb/teams%zu/wg%lld/S%d", qt.size(), wg,
                          a->steps < 1000 ? a->steps : 1000);
            if (!hsb::tune_lookup(key, &policy) || policy > 1) {
                policy = 0;
                if (cap == hipStreamCaptureStatusNone) {
                    hsb::QRun tr = qr;
                    tr.steps = std::min(a->steps, 200);
                    std::vector<double> ms(2, 0.0);
                    hipEvent_t e0 = nullptr, e1 = nullptr;
                    HIP_TRY(hipEventCreate(&e0));
                    HIP_TRY(hipEventCreate(&e1));
                    hsb::KernelTimer off;
                    int trc = HSB_OK;
                    for (int v = 0; v < 2 && trc == HSB_OK; ++v)
                        for (int rep = 0; rep < 2 && trc == HSB_OK; ++rep) {
                            float f = 0.0f;
                            hipError_t he = hipEventRecord(e0, s);
                            if (he == hipSuccess) trc = hsb::queue_run(lead->qwork, qt, tr, v, s, off);
                            if (trc == HSB_OK && he == hipSuccess) he = hipEventRecord(e1, s);
                            if (trc == HSB_OK && he == hipSuccess) he = hipEventSynchronize(e1);
                            if (trc == HSB_OK && he == hipSuccess) he = hipEventElapsedTime(&f, e0, e1);
                            if (trc == HSB_OK && he != hipSuccess) trc = hip_fail(he, "timing a policy");
                            ms[v] = f;
                        }
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    if (trc != HSB_OK) return trc == HSB_EDEVICE ? trc : fail(trc, "%s", hsb::queue_error());
                    policy = ms[1] < ms[0] ? 1 : 0;
                    (void)hsb::tune_store(key, policy, ms);
                }
            }
        }
        const bool graphable = lead->graph && !lead->timing && singles.empty() &&
                               classes.empty() && cap == hipStreamCaptureStatusNone;
        int rc;
        if (graphable) {
            rc = batch_graph(lead, qt, qr, s, policy);
        } else {
            batch_graph_drop(lead);
            rc = hsb::queue_run(lead->qwork, qt, qr, policy, s, lead->timer);
            if (rc != HSB_OK) rc = fail(rc, "%s", hsb::queue_error());
        }
        lead->last_tile = policy;
        if (rc != HSB_OK) return rc;
        int32_t status = 0;
        HIP_TRY(hipMemcpyAsync(&status, hsb::queue_status(lead->qwork), sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (status & 2) return fail(HSB_EDEVICE, "batch queue kernel: exchange wait timed out");
        any_bad |= status & 1;
        lead->last_plan = PLAN_FP4;
    }
    // the rest: one persistent launch sequence per padded size
    // The classes' state: kept by the lead context and grown only when a class
    // needs more elements or columns than it holds (the FP4 plan uses neither
    // the FP32 operand nor its energy buffers).  Class c uses Nst Rtot elements
    // with leading dimension Rtot.
    {
        size_t need_ns = 0, need_nr = 0;
        for (auto &cls : classes) {
            size_t cols = 0;
            for (int j : cls.second) cols += (size_t)round_up(jobs[j].R, 32);
            const size_t rtot = (size_t)round_up((int)cols, hsb::kTile);
            need_ns = std::max(need_ns, (size_t)cls.first * 64 * rtot);
            need_nr = std::max(need_nr, rtot);
        }
        if (need_ns > lead->bstate_ns || need_nr > lead->bstate_nr) {
            hsb::free_state_bufs(lead->bstate);
            lead->bstate_ns = lead->bstate_nr = 0;
            const int rows = (int)((need_ns + need_nr - 1) / need_nr);
            hipError_t ea = hsb::alloc_state(lead->bstate, rows, (int)need_nr, false);
            if (ea != hipSuccess) return hip_fail(ea, "allocating batch state");
            lead->bstate_ns = (size_t)rows * need_nr;
            lead->bstate_nr = need_nr;
        }
    }
    for (auto &cls : classes) {
        const int nkb = cls.first, Nst = nkb * 64;
        const std::vector<int> &cj = cls.second;
        // columns: job j owns [col0, col0 + round_up(R, 32)), 32-replica teams
        std::vector<int> col0(cj.size());
        int used = 0;
        for (size_t q = 0; q < cj.size(); ++q) {
            col0[q] = used;
            used += round_up(jobs[cj[q]].R, 32);
        }
        const int Rtot = round_up(used, hsb::kTile);
        std::vector<hsb::FP4Team> teams;
        for (size_t q = 0; q < cj.size(); ++q) {
            const hsb_job &jb = jobs[cj[q]];
            hsb_ctx *h = hs[jb.instance];
            if (!h->pj) {
                const int rc = hsb::persistent_create(h->hJ.data(), h->N, &h->pj);
                if (rc != HSB_OK) return fail(rc, "%s", hsb::persistent_error());
            }
            for (int t = 0; t < round_up(jb.R, 32) / 32; ++t)
                teams.push_back(hsb::FP4Team{hsb::persistent_jpk(h->pj), h->N, jb.c0});
        }
        if (!lead->bwork) {
            const int rc = hsb::persistent_work_create(&lead->bwork);
            if (rc != HSB_OK) return fail(rc, "%s", hsb::persistent_error());
        }
        hsb::StateBufs &bb = lead->bstate;  // sized for every class above
        // the class's job table (device copy read by the set-up and output kernels)
        std::vector<hsb::BatchJob> bj(cj.size());
        int Nmax = 0;
        for (size_t q = 0; q < cj.size(); ++q) {
            const hsb_job &jb = jobs[cj[q]];
            bj[q] = hsb::BatchJob{col0[q], jb.R, hs[jb.instance]->N, jb.gamma, jb.seed, jb.spins,
                                  jb.energy};
            if (bj[q].N > Nmax) Nmax = bj[q].N;
        }
        if (bj.size() > lead->bjobs_cap) {
            if (lead->bjobs) (void)hipFree(lead->bjobs);
            lead->bjobs = nullptr;
            lead->bjobs_cap = 0;
            HIP_TRY(hipMalloc((void **)&lead->bjobs, sizeof(hsb::BatchJob) * bj.size()));
            lead->bjobs_cap = bj.size();
        }
        auto done = [&](int rc) {
            (void)hipStreamSynchronize(s);  // also keeps bj alive until its copy is done
            return rc;
        };
        hipError_t e = hipMemcpyAsync(lead->bjobs, bj.data(), sizeof(hsb::BatchJob) * bj.size(),
                                      hipMemcpyHostToDevice, s);
        // initial state and gamma per column (zero columns between jobs), tracking
        if (e == hipSuccess)
            e = hsb::launch_init_batch(bb.X, bb.Y, bb.gamma, lead->bjobs, (int)bj.size(), Nst, Rtot,
                                       (float)amp, s);
        if (e == hipSuccess) e = hsb::launch_reset_tracking(bb, Rtot, s);
        if (e != hipSuccess) return done(hip_fail(e, "batch set-up"));
        hsb::PersistentRun pr{};
        pr.X = bb.X; pr.Y = bb.Y; pr.gamma = bb.gamma;
        pr.Npad = Nst; pr.Rpad = Rtot; pr.R = used;
        pr.k0 = 0; pr.k1 = a->steps; pr.Ns = a->steps; pr.interval = interval;
        pr.a0 = a->a0; pr.c0 = 0.0f; pr.dt = a->dt;
        pr.local_exchange = hs[0]->local_exchange;
        int rc = hsb::persistent_run_teams(lead->bwork, a->variant, nkb, teams.data(),
                                           (int)teams.size(), pr, bb, Nst, s, lead->timer);
        if (rc != HSB_OK) return done(fail(rc, "%s", hsb::persistent_error()));
        e = hsb::launch_output_batch(bb, lead->bjobs, (int)bj.size(), Nmax, Rtot, a->return_best, s);
        int32_t status = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&status, bb.status, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return done(hip_fail(e, "batch output"));
        if (status & 2)
            return done(fail(HSB_EDEVICE, "FP4 persistent kernel: exchange wait timed out"));
        any_bad |= status;
        done(HSB_OK);
        lead->last_plan = PLAN_FP4;
    }

    if (any_bad) return fail(HSB_ENUMERIC, "a replica's state became non-finite");
    return HSB_OK;
}
