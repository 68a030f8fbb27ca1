// C ABI of the correlator: argument validation, the plan (buffer sizes and
// the device-memory budget), integration state, and the launches.
//
// Validation always runs before the first HIP call of a function, so every
// invalid-argument, budget and overflow error is decided on the CPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "corr.h"
#include "corr_internal.h"

using namespace corr;

struct corr_ctx {
    corr_params p{};
    int N = 0, C = 0, prec = 0, TB = 0, n_tb_cap = 0;
    SpecLayout lay{};                 // strides of the spectra buffer
    bool tb_major = false;            // its order (time-block-major or channel-major)
    std::string arch;                 // the device's architecture name (tuning cache key)
    int num_cus = 256;                // compute units of the device
    int64_t B = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    void *spec = nullptr;
    size_t spec_bytes = 0;
    void *acc = nullptr;
    size_t acc_bytes = 0;
    float2 *twiddle = nullptr;
    float2 *twiddle2n = nullptr;       // exp(-j pi k / C), k < C (real-input F-engine)
    float *unit_scale = nullptr;       // C ones: the F-engine's scale when the caller gives none
    void *gscr = nullptr;             // F-engine chunk scratch (kGatherMinC channels and up)
    int64_t gscr_bytes = 0;
    bool owns_gscr = true;            // false: the batch's shared scratch
    float *scale2 = nullptr;          // s_k^2 of the F-engine's spectra
    float *scale2_user = nullptr;     // s_k^2 of caller spectra
    void *dump_tmp = nullptr;         // staging for converted dumps to host
    int n_held = 0;                   // spectra in the buffer
    bool held_from_fengine = false;
    int64_t n_integrated = 0;         // spectra integrated since the last reset
    bool acc_zero = true;             // accumulators logically zero
    int tile = 0;                     // X-engine block size; 0 = by N
    bool batch_member = false;        // owned by a corr_batch
    int *zflag = nullptr;             // batch members: device "zero since reset" flag
    std::string err;
};

struct corr_batch {
    std::vector<corr_ctx *> subs;
    int prec = 0;
    hipStream_t stream = nullptr;
    int num_cus = 0;                  // compute units of the device
    uint8_t *d_plan = nullptr;        // device work plan: XQueue[2], then XDesc[n]
    uint8_t *h_plan = nullptr;        // pinned staging of the plan
    std::vector<uint8_t> last;        // plan last uploaded
    unsigned int *d_counter = nullptr;  // per-XCD work counters of both block-size groups
    void *d_gscr = nullptr;           // F-engine scratch shared by the sub-arrays (one stream)
    int *d_zflag = nullptr;           // one "zero since reset" flag per sub-array
    std::string err;
};

namespace {

thread_local std::string g_err;
// Set while corr_create_batched creates its sub-arrays: they share one
// F-engine scratch owned by the batch instead of each allocating its own.
thread_local bool g_no_own_scratch = false;

corr_status fail(corr_ctx *h, corr_status s, const std::string &msg) {
    if (h)
        h->err = msg;
    else
        g_err = msg;
    return s;
}

corr_status hip_fail(corr_ctx *h, hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(h, e == hipErrorOutOfMemory ? CORR_E_NOMEM : CORR_E_HIP, m);
}

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Validates params; fills N, B, C, prec on success.  No HIP calls.
corr_status check_params(const corr_params *p, std::string &msg) {
    if (!p) {
        msg = "params is NULL";
        return CORR_E_INVALID_ARG;
    }
    if (p->n_stations < 1) {
        msg = "n_stations must be >= 1";
        return CORR_E_INVALID_ARG;
    }
    if (p->n_pols != 1 && p->n_pols != 2) {
        msg = "n_pols must be 1 or 2";
        return CORR_E_INVALID_ARG;
    }
    if (!is_pow2(p->n_channels)) {
        msg = "n_channels must be a power of two";
        return CORR_E_INVALID_ARG;
    }
    if (p->n_channels < CORR_MIN_CHANNELS || p->n_channels > CORR_MAX_CHANNELS) {
        msg = "n_channels outside 16..8192";
        return CORR_E_UNSUPPORTED;
    }
    if (p->n_integrate < 1) {
        msg = "n_integrate must be >= 1";
        return CORR_E_INVALID_ARG;
    }
    if (p->precision < CORR_FP32 || p->precision > CORR_INT8) {
        msg = "unknown precision";
        return CORR_E_INVALID_ARG;
    }
    if (p->layout < CORR_TRI_LOWER || p->layout > CORR_FULL) {
        msg = "unknown layout";
        return CORR_E_INVALID_ARG;
    }
    if (p->order < CORR_CHAN_MAJOR || p->order > CORR_BASELINE_MAJOR) {
        msg = "unknown order";
        return CORR_E_INVALID_ARG;
    }
    if (p->reserved != 0) {
        msg = "reserved must be 0";
        return CORR_E_INVALID_ARG;
    }
    const int64_t N = (int64_t)p->n_stations * p->n_pols;
    if (N > CORR_MAX_INPUTS) {
        msg = "more than 8192 inputs";
        return CORR_E_UNSUPPORTED;
    }
    if (p->precision == CORR_INT8 && p->n_integrate > CORR_INT8_MAX_INTEGRATE) {
        msg = "int8 integration longer than 66572 spectra could overflow int32";
        return CORR_E_OVERFLOW;
    }
    return CORR_OK;
}

int64_t n_inputs(const corr_params *p) { return (int64_t)p->n_stations * p->n_pols; }

int64_t layout_products(const corr_params *p) {
    const int64_t N = n_inputs(p);
    return p->layout == CORR_FULL ? N * N : N * (N + 1) / 2;
}

bool default_dump(const corr_params *p) { return p->layout == CORR_TRI_LOWER && p->order == CORR_CHAN_MAJOR; }

bool aligned(const void *ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

// Default block size when none was set or tuned, from measured X-engine
// speed on MI355X at 256..1024 inputs: 64-input blocks (four workgroups per
// CU) win for FP32, 128-input blocks (eight 64x32 waves, more operand reuse)
// for the FP16, int8 and FP8 forms.
int effective_tile(const corr_ctx *h) {
    if (h->tile) return h->tile;
    return (h->N <= 64 || h->prec == P_FP32) ? 64 : 128;
}

const float *x_scale(const corr_ctx *h) {
    if (h->prec == P_INT8) return nullptr;
    if (h->held_from_fengine) return h->scale2;
    return h->prec == P_FP32 ? nullptr : h->scale2_user;
}

// Autotune cache.  Key: the device's architecture name, the precision, the
// inputs rounded up to 64 (the smaller block size), the channels, the time
// blocks timed and (for the X-engine-only tuner) the spectra order; value:
// the block size and, for the F + X tuner, the spectra order.  Kept for the
// process and, when CORR_TUNE_CACHE names a file, appended to it as lines
//   fx <arch> <prec> <N/64> <C> <n_tb> <tile> <tb_major>
//   x  <arch> <prec> <N/64> <C> <n_tb> <tb_major> <tile>
// (other lines are ignored).
struct TuneKey {
    std::string arch;
    int kind, prec, nb, C, n_tb, order;       // kind 0: X-engine only, 1: F + X
    bool operator<(const TuneKey &o) const {
        return std::tie(arch, kind, prec, nb, C, n_tb, order) < std::tie(o.arch, o.kind, o.prec, o.nb, o.C, o.n_tb, o.order);
    }
};
struct TuneVal {
    int tile, tb_major;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
bool g_tune_loaded = false;

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("CORR_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512], kind[8], arch[128];
    while (std::fgets(line, sizeof line, f)) {
        int p, nb, C, nt, v1, v2;
        if (std::sscanf(line, "%7s %127s %d %d %d %d %d %d", kind, arch, &p, &nb, &C, &nt, &v1, &v2) != 8) continue;
        if (!std::strcmp(kind, "fx") && (v1 == 64 || v1 == 128) && (v2 == 0 || v2 == 1))
            g_tune[{arch, 1, p, nb, C, nt, 0}] = {v1, v2};
        else if (!std::strcmp(kind, "x") && (v1 == 0 || v1 == 1) && (v2 == 64 || v2 == 128))
            g_tune[{arch, 0, p, nb, C, nt, v1}] = {v2, v1};
    }
    std::fclose(f);
}

void tune_store_locked(const TuneKey &k, TuneVal v) {
    g_tune[k] = v;
    const char *path = std::getenv("CORR_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    if (k.kind == 1)
        std::fprintf(f, "fx %s %d %d %d %d %d %d\n", k.arch.c_str(), k.prec, k.nb, k.C, k.n_tb, v.tile, v.tb_major);
    else
        std::fprintf(f, "x %s %d %d %d %d %d %d\n", k.arch.c_str(), k.prec, k.nb, k.C, k.n_tb, k.order, v.tile);
    std::fclose(f);
}

// Channels an autotuner times the X-engine on: at least 256, and enough that
// both block sizes give four workgroups per slot the GPU holds (two of 128
// inputs or four of 64 per CU), so a small array is timed at throughput, not
// at the latency of a launch that leaves the GPU half empty.
int tune_channels(const corr_ctx *h) {
    const int64_t nb = (h->N + 127) / 128;
    const int64_t tiles128 = nb * (nb + 1) / 2;
    const int64_t need = (4 * 2 * (int64_t)h->num_cus + tiles128 - 1) / tiles128;
    return (int)std::min<int64_t>(h->C, std::max<int64_t>(256, need));
}

// An autotuner replaces the built-in choice only by a candidate at least 2%
// faster: the two block sizes often time within a percent of each other on
// the channel subset, and which wins there need not win on all channels
// (1024 inputs x 4096 FP32 channels: 64-input blocks 137.1-137.5 ms, 128-input
// blocks 137.7-138.1 ms in full, the reverse on 256 channels).
constexpr float kTuneMargin = 0.98f;

// Timing events and a scratch buffer owned by an autotuner call.
struct TuneScope {
    hipEvent_t ev[3] = {};
    int n_ev = 0;
    void *tmp = nullptr;
    hipError_t create(int n_events, size_t tmp_bytes) {
        for (n_ev = 0; n_ev < n_events; ++n_ev) {
            const hipError_t e = hipEventCreate(&ev[n_ev]);
            if (e != hipSuccess) return e;
        }
        return hipMalloc(&tmp, tmp_bytes);
    }
    ~TuneScope() {
        for (int i = 0; i < n_ev; ++i) (void)hipEventDestroy(ev[i]);
        if (tmp) (void)hipFree(tmp);
    }
};

// The device's architecture name (gcnArchName, e.g. "gfx950:sramecc+:xnack-").
std::string device_arch(int dev) {
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    for (char &c : a)
        if (c == ' ') c = '_';
    return a.empty() ? "unknown" : a;
}

}  // namespace

static void destroy_ctx(corr_ctx *h);

extern "C" {

int64_t corr_n_products(const corr_params *params) {
    std::string m;
    if (check_params(params, m) != CORR_OK) return -1;
    const int64_t N = n_inputs(params);
    return N * (N + 1) / 2;
}

int64_t corr_visibility_bytes(const corr_params *params) {
    std::string m;
    if (check_params(params, m) != CORR_OK) return -1;
    return layout_products(params) * params->n_channels * 8;
}

int64_t corr_spectra_bytes(const corr_params *params, int32_t n_spectra) {
    std::string m;
    if (check_params(params, m) != CORR_OK || n_spectra < 0) return -1;
    return (int64_t)n_spectra * params->n_channels * n_inputs(params) * 2 * elem_bytes(params->precision);
}

const char *corr_status_string(corr_status s) {
    switch (s) {
    case CORR_OK: return "CORR_OK";
    case CORR_E_INVALID_ARG: return "CORR_E_INVALID_ARG: invalid argument";
    case CORR_E_UNSUPPORTED: return "CORR_E_UNSUPPORTED: unsupported configuration";
    case CORR_E_NOMEM: return "CORR_E_NOMEM: device memory budget exceeded";
    case CORR_E_OVERFLOW: return "CORR_E_OVERFLOW: int8 integration could overflow int32";
    case CORR_E_STATE: return "CORR_E_STATE: call out of order";
    case CORR_E_HIP: return "CORR_E_HIP: HIP runtime error";
    default: return "unknown corr_status";
    }
}

const char *corr_last_error(corr_handle h) { return h ? h->err.c_str() : g_err.c_str(); }

corr_status corr_create(const corr_params *params, void *hip_stream, corr_handle *out) {
    std::string msg;
    corr_status s = check_params(params, msg);
    if (s != CORR_OK) return fail(nullptr, s, msg);
    if (!out) return fail(nullptr, CORR_E_INVALID_ARG, "out is NULL");

    const int N = (int)n_inputs(params);
    const int C = params->n_channels;
    const int prec = params->precision;
    const int TB = time_block(prec);
    const int n_tb_cap = (params->n_integrate + TB - 1) / TB;
    const size_t spec_bytes = (size_t)spec_buffer_bytes(C, N, n_tb_cap, elem_bytes(prec));
    const int64_t B = (int64_t)N * (N + 1) / 2;
    const size_t acc_bytes = (size_t)C * B * 8;
    const size_t small_bytes = (size_t)C * 8 + 2 * (size_t)C * 4;
    const size_t dump_bytes = default_dump(params) ? 0 : (size_t)corr_visibility_bytes(params);
    const size_t gscr_bytes = g_no_own_scratch ? 0 : (size_t)gather_scratch_bytes(C, N, n_tb_cap);
    const size_t need = spec_bytes + acc_bytes + small_bytes + dump_bytes + gscr_bytes;
    if (params->device_mem_cap && need > params->device_mem_cap) {
        char b[160];
        snprintf(b, sizeof b, "plan needs %zu bytes, cap is %llu", need,
                 (unsigned long long)params->device_mem_cap);
        return fail(nullptr, CORR_E_NOMEM, b);
    }

    // ---- HIP from here on ----
    corr_ctx *h = new (std::nothrow) corr_ctx();
    if (!h) return fail(nullptr, CORR_E_NOMEM, "host allocation failed");
    h->p = *params;
    h->N = N;
    h->C = C;
    h->prec = prec;
    h->TB = TB;
    h->n_tb_cap = n_tb_cap;
    h->tb_major = default_tb_major(C, N, elem_bytes(prec));
    h->lay = spec_layout_of(C, N, n_tb_cap, h->tb_major);
    h->B = B;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->spec_bytes = spec_bytes;
    h->acc_bytes = acc_bytes;

    auto cleanup_fail = [&](corr_status st, const std::string &m) {
        g_err = m;
        destroy_ctx(h);
        return st;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        std::string m = std::string("hipGetDevice: ") + hipGetErrorString(e);
        delete h;
        return fail(nullptr, CORR_E_HIP, m);
    }
    h->arch = device_arch(h->device);
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cus > 0)
            h->num_cus = cus;
    }
    if (!params->device_mem_cap) {
        size_t fr = 0, tot = 0;
        e = hipMemGetInfo(&fr, &tot);
        if (e != hipSuccess) {
            std::string m = std::string("hipMemGetInfo: ") + hipGetErrorString(e);
            delete h;
            return fail(nullptr, CORR_E_HIP, m);
        }
        if (need > fr) {
            char b[160];
            snprintf(b, sizeof b, "plan needs %zu bytes, device has %zu free", need, fr);
            delete h;
            return fail(nullptr, CORR_E_NOMEM, b);
        }
    }
    if ((e = hipMalloc(&h->spec, spec_bytes)) != hipSuccess)
        return cleanup_fail(e == hipErrorOutOfMemory ? CORR_E_NOMEM : CORR_E_HIP, "hipMalloc spectra failed");
    if ((e = hipMalloc(&h->acc, acc_bytes)) != hipSuccess)
        return cleanup_fail(e == hipErrorOutOfMemory ? CORR_E_NOMEM : CORR_E_HIP, "hipMalloc accumulators failed");
    if (gscr_bytes && (e = hipMalloc(&h->gscr, gscr_bytes)) != hipSuccess)
        return cleanup_fail(e == hipErrorOutOfMemory ? CORR_E_NOMEM : CORR_E_HIP, "hipMalloc F-engine scratch failed");
    h->gscr_bytes = (int64_t)gscr_bytes;
    if ((e = hipMalloc(&h->twiddle, (size_t)C * sizeof(float2))) != hipSuccess ||
        (e = hipMalloc(&h->twiddle2n, (size_t)C * sizeof(float2))) != hipSuccess ||
        (e = hipMalloc(&h->unit_scale, (size_t)C * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&h->scale2, (size_t)C * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&h->scale2_user, (size_t)C * sizeof(float))) != hipSuccess)
        return cleanup_fail(CORR_E_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));

    // Twiddles W[m] = exp(-j 2 pi m / C), computed in float64, rounded to float32.
    // W2[k] = exp(-j 2 pi k / 2C) for the real-input split, the same way.
    std::vector<float2> tw(C), tw2(C);
    const double two_pi = 6.283185307179586476925286766559;
    for (int m = 0; m < C; ++m) {
        const double ang = two_pi * (double)m / (double)C;
        tw[m] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
        const double ang2 = two_pi * (double)m / (2.0 * (double)C);
        tw2[m] = make_float2((float)std::cos(ang2), (float)-std::sin(ang2));
    }
    if ((e = hipMemcpy(h->twiddle, tw.data(), (size_t)C * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(h->twiddle2n, tw2.data(), (size_t)C * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(h->unit_scale, std::vector<float>(C, 1.0f).data(), (size_t)C * sizeof(float),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup_fail(CORR_E_HIP, std::string("hipMemcpy twiddles: ") + hipGetErrorString(e));
    *out = h;
    return CORR_OK;
}

}  // extern "C"

static void destroy_ctx(corr_ctx *h) {
    if (h->spec || h->acc) (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->spec);
    (void)hipFree(h->acc);
    (void)hipFree(h->twiddle);
    (void)hipFree(h->twiddle2n);
    (void)hipFree(h->unit_scale);
    if (h->owns_gscr) (void)hipFree(h->gscr);
    (void)hipFree(h->scale2);
    (void)hipFree(h->scale2_user);
    (void)hipFree(h->dump_tmp);
    delete h;
}

extern "C" {

corr_status corr_destroy(corr_handle h) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (h->batch_member) return fail(h, CORR_E_STATE, "sub-array handles are destroyed with their batch");
    destroy_ctx(h);
    return CORR_OK;
}

}  // extern "C"

// Placement checks shared by the F-engine entry points: spectra
// [first, first + n) of the held set, first a whole number of time blocks and
// no gap after the spectra already held.
static corr_status check_placement(corr_ctx *h, int32_t first, int32_t n_spectra) {
    if (first < 0) return fail(h, CORR_E_INVALID_ARG, "first_spectrum must be >= 0");
    if (first % time_block(h->prec))
        return fail(h, CORR_E_INVALID_ARG, "first_spectrum must be a multiple of the time block");
    if (n_spectra < 1 || (int64_t)first + n_spectra > h->p.n_integrate)
        return fail(h, CORR_E_INVALID_ARG, "need 1 <= n_spectra and first_spectrum + n_spectra <= n_integrate");
    if (first > 0 && (!h->held_from_fengine || first > h->n_held))
        return fail(h, CORR_E_STATE, "appending needs F-engine spectra held up to first_spectrum");
    return CORR_OK;
}

extern "C" {

corr_status corr_fengine_at(corr_handle h, const void *d_volts, int64_t ld_samples, int32_t n_spectra,
                            const float *d_inv_scale, int32_t first_spectrum) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (!d_volts) return fail(h, CORR_E_INVALID_ARG, "d_volts is NULL");
    if (!aligned(d_volts, 8)) return fail(h, CORR_E_INVALID_ARG, "d_volts must be 8-byte aligned");
    if (d_inv_scale && !aligned(d_inv_scale, 4)) return fail(h, CORR_E_INVALID_ARG, "d_inv_scale misaligned");
    corr_status st = check_placement(h, first_spectrum, n_spectra);
    if (st != CORR_OK) return st;
    if (ld_samples < (int64_t)n_spectra * h->C)
        return fail(h, CORR_E_INVALID_ARG, "ld_samples < n_spectra * n_channels");
    if (h->prec == P_INT8 && !d_inv_scale)
        return fail(h, CORR_E_INVALID_ARG, "int8 needs a per-channel scale");

    hipError_t e = launch_scale2(h->C, d_inv_scale, h->scale2, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "scale2 launch");
    e = launch_fengine(h->prec, h->C, h->N, static_cast<const float2 *>(d_volts), ld_samples, n_spectra,
                       d_inv_scale ? d_inv_scale : h->unit_scale, h->twiddle, h->spec, h->lay,
                       FScratch{h->gscr, h->gscr_bytes}, first_spectrum / time_block(h->prec), h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "fengine launch");
    h->n_held = first_spectrum + n_spectra;
    h->held_from_fengine = true;
    h->err.clear();
    return CORR_OK;
}

corr_status corr_fengine(corr_handle h, const void *d_volts, int64_t ld_samples, int32_t n_spectra,
                         const float *d_inv_scale) {
    return corr_fengine_at(h, d_volts, ld_samples, n_spectra, d_inv_scale, 0);
}

corr_status corr_fengine_real8_at(corr_handle h, const int8_t *d_samples, int64_t ld_samples, int32_t n_spectra,
                                  const float *d_inv_scale, int32_t first_spectrum) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (!d_samples) return fail(h, CORR_E_INVALID_ARG, "d_samples is NULL");
    if (!aligned(d_samples, 2)) return fail(h, CORR_E_INVALID_ARG, "d_samples must be 2-byte aligned");
    if (ld_samples % 2) return fail(h, CORR_E_INVALID_ARG, "ld_samples must be even");
    if (d_inv_scale && !aligned(d_inv_scale, 4)) return fail(h, CORR_E_INVALID_ARG, "d_inv_scale misaligned");
    corr_status st = check_placement(h, first_spectrum, n_spectra);
    if (st != CORR_OK) return st;
    if (ld_samples < (int64_t)n_spectra * 2 * h->C)
        return fail(h, CORR_E_INVALID_ARG, "ld_samples < n_spectra * 2 * n_channels");
    if (h->prec == P_INT8 && !d_inv_scale)
        return fail(h, CORR_E_INVALID_ARG, "int8 needs a per-channel scale");

    hipError_t e = launch_scale2(h->C, d_inv_scale, h->scale2, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "scale2 launch");
    e = launch_fengine_real8(h->prec, h->C, h->N, d_samples, ld_samples, n_spectra,
                             d_inv_scale ? d_inv_scale : h->unit_scale, h->twiddle, h->twiddle2n, h->spec,
                             h->lay, FScratch{h->gscr, h->gscr_bytes}, first_spectrum / time_block(h->prec), h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "fengine_real8 launch");
    h->n_held = first_spectrum + n_spectra;
    h->held_from_fengine = true;
    h->err.clear();
    return CORR_OK;
}

corr_status corr_fengine_real8(corr_handle h, const int8_t *d_samples, int64_t ld_samples, int32_t n_spectra,
                               const float *d_inv_scale) {
    return corr_fengine_real8_at(h, d_samples, ld_samples, n_spectra, d_inv_scale, 0);
}

}  // extern "C"

extern "C" {

corr_status corr_fx(corr_handle h, const void *d_volts, int64_t ld_samples, int32_t n_spectra,
                    const float *d_inv_scale, int32_t chunk_spectra) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (!d_volts || !aligned(d_volts, 8)) return fail(h, CORR_E_INVALID_ARG, "d_volts must be 8-byte aligned");
    if (d_inv_scale && !aligned(d_inv_scale, 4)) return fail(h, CORR_E_INVALID_ARG, "d_inv_scale misaligned");
    if (n_spectra < 1) return fail(h, CORR_E_INVALID_ARG, "n_spectra must be >= 1");
    if (chunk_spectra < 1 || chunk_spectra % h->TB || chunk_spectra > h->p.n_integrate)
        return fail(h, CORR_E_INVALID_ARG,
                    "chunk_spectra must be a multiple of the time block and at most n_integrate");
    if (ld_samples < (int64_t)n_spectra * h->C)
        return fail(h, CORR_E_INVALID_ARG, "ld_samples < n_spectra * n_channels");
    if (h->prec == P_INT8 && !d_inv_scale) return fail(h, CORR_E_INVALID_ARG, "int8 needs a per-channel scale");
    if (h->batch_member) return fail(h, CORR_E_STATE, "sub-array handles integrate with corr_xengine_batched");
    if (h->prec == P_INT8 && h->n_integrated + n_spectra > CORR_INT8_MAX_INTEGRATE)
        return fail(h, CORR_E_OVERFLOW, "int8 integration would exceed 66572 spectra since the last reset");

    hipError_t e = launch_scale2(h->C, d_inv_scale, h->scale2, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "scale2 launch");
    const float2 *v = static_cast<const float2 *>(d_volts);
    int last = 0;
    for (int32_t s0 = 0; s0 < n_spectra; s0 += chunk_spectra) {
        const int ns = std::min(chunk_spectra, n_spectra - s0);
        e = launch_fengine(h->prec, h->C, h->N, v + (int64_t)s0 * h->C, ld_samples, ns,
                           d_inv_scale ? d_inv_scale : h->unit_scale, h->twiddle, h->spec, h->lay,
                           FScratch{h->gscr, h->gscr_bytes}, 0, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "fengine launch");
        e = launch_xengine(h->prec, effective_tile(h), h->C, h->N, ns, h->spec, h->lay,
                           h->prec == P_INT8 ? nullptr : h->scale2, h->acc, h->acc, h->acc_zero ? 1 : 0, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "xengine launch");
        h->acc_zero = false;
        last = ns;
    }
    h->n_held = last;
    h->held_from_fengine = true;
    h->n_integrated += n_spectra;
    h->err.clear();
    return CORR_OK;
}

}  // extern "C"

// Checks of an X-engine call, the ingest of caller spectra, and the scale the
// X-engine applies (shared by corr_xengine and corr_xengine_dump).
static corr_status prepare_x(corr_ctx *h, const void *d_spectra, int32_t n_spectra, const float *d_inv_scale,
                             const float **s2_out) {
    if (n_spectra < 1) return fail(h, CORR_E_INVALID_ARG, "n_spectra must be >= 1");
    if (d_spectra) {
        if (!aligned(d_spectra, 16)) return fail(h, CORR_E_INVALID_ARG, "d_spectra must be 16-byte aligned");
        if (n_spectra > h->p.n_integrate) return fail(h, CORR_E_INVALID_ARG, "n_spectra > n_integrate");
        if (d_inv_scale && (h->prec == P_FP32 || h->prec == P_INT8))
            return fail(h, CORR_E_INVALID_ARG, "d_inv_scale applies only to FP16/FP8 caller spectra");
        if (d_inv_scale && !aligned(d_inv_scale, 4)) return fail(h, CORR_E_INVALID_ARG, "d_inv_scale misaligned");
    } else {
        if (d_inv_scale) return fail(h, CORR_E_INVALID_ARG, "d_inv_scale must be NULL for held spectra");
        if (h->n_held == 0) return fail(h, CORR_E_STATE, "no spectra held: call corr_fengine first");
        if (n_spectra > h->n_held) return fail(h, CORR_E_STATE, "n_spectra exceeds the spectra held");
    }
    if (h->prec == P_INT8 && h->n_integrated + n_spectra > CORR_INT8_MAX_INTEGRATE)
        return fail(h, CORR_E_OVERFLOW, "int8 integration would exceed 66572 spectra since the last reset");

    hipError_t e;
    const float *s2 = nullptr;
    if (d_spectra) {
        e = launch_ingest(h->prec, h->C, h->N, n_spectra, h->lay, d_spectra, h->spec, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "ingest launch");
        h->n_held = n_spectra;
        h->held_from_fengine = false;
        if (h->prec == P_FP16 || h->prec == P_FP8) {
            e = launch_scale2(h->C, d_inv_scale, h->scale2_user, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "scale2 launch");
            s2 = h->scale2_user;
        }
    } else {
        s2 = x_scale(h);
    }
    *s2_out = s2;
    return CORR_OK;
}

extern "C" {

corr_status corr_xengine(corr_handle h, const void *d_spectra, int32_t n_spectra, const float *d_inv_scale) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    const float *s2 = nullptr;
    const corr_status st = prepare_x(h, d_spectra, n_spectra, d_inv_scale, &s2);
    if (st != CORR_OK) return st;
    hipError_t e = launch_xengine(h->prec, effective_tile(h), h->C, h->N, n_spectra, h->spec, h->lay, s2, h->acc,
                                  h->acc, h->acc_zero ? 1 : 0, h->stream, h->zflag);
    if (e == hipSuccess && h->zflag) e = launch_set_flag(h->zflag, 0, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "xengine launch");
    h->acc_zero = false;
    h->n_integrated += n_spectra;
    h->err.clear();
    return CORR_OK;
}

corr_status corr_xengine_dump(corr_handle h, const void *d_spectra, int32_t n_spectra, const float *d_inv_scale,
                              void *d_dst) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (!d_dst || !aligned(d_dst, 8)) return fail(h, CORR_E_INVALID_ARG, "d_dst must be an 8-byte aligned device pointer");
    if (!default_dump(&h->p))
        return fail(h, CORR_E_UNSUPPORTED, "the fused dump writes the lower-triangle, channel-major layout only");
    if (h->batch_member) return fail(h, CORR_E_STATE, "sub-array handles integrate with corr_xengine_batched");
    const float *s2 = nullptr;
    const corr_status st = prepare_x(h, d_spectra, n_spectra, d_inv_scale, &s2);
    if (st != CORR_OK) return st;
    const hipError_t e = launch_xengine(h->prec, effective_tile(h), h->C, h->N, n_spectra, h->spec, h->lay, s2,
                                        d_dst, h->acc, h->acc_zero ? 1 : 0, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "xengine launch");
    h->acc_zero = true;                                  // the integration ends here: reset
    h->n_integrated = 0;
    h->err.clear();
    return CORR_OK;
}

corr_status corr_xengine_rect(corr_handle h, int32_t i0, int32_t ni, int32_t j0, int32_t nj, int32_t n_spectra,
                              void *d_out, int32_t accumulate) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (ni < 1 || nj < 1 || i0 < 0 || j0 < 0 || (int64_t)i0 + ni > h->N || (int64_t)j0 + nj > h->N)
        return fail(h, CORR_E_INVALID_ARG, "row and column ranges must be non-empty and within the inputs");
    if (!((int64_t)i0 + ni <= j0 || (int64_t)j0 + nj <= i0))
        return fail(h, CORR_E_INVALID_ARG, "row and column ranges overlap: use corr_xengine for a triangle");
    if (!d_out || !aligned(d_out, 8)) return fail(h, CORR_E_INVALID_ARG, "d_out must be an 8-byte aligned device pointer");
    if (accumulate != 0 && accumulate != 1) return fail(h, CORR_E_INVALID_ARG, "accumulate must be 0 or 1");
    if (n_spectra < 1) return fail(h, CORR_E_INVALID_ARG, "n_spectra must be >= 1");
    if (h->n_held == 0) return fail(h, CORR_E_STATE, "no spectra held: call corr_fengine first");
    if (n_spectra > h->n_held) return fail(h, CORR_E_STATE, "n_spectra exceeds the spectra held");
    if (h->prec == P_INT8 && n_spectra > CORR_INT8_MAX_INTEGRATE)
        return fail(h, CORR_E_OVERFLOW, "int8 rectangle over more than 66572 spectra");
    const hipError_t e = launch_xengine_rect(h->prec, effective_tile(h), h->C, h->N, n_spectra, h->spec,
                                             h->lay, x_scale(h), d_out, accumulate ? 0 : 1, i0, ni, j0, nj,
                                             h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "rectangle launch");
    h->err.clear();
    return CORR_OK;
}

corr_status corr_dump_visibilities(corr_handle h, void *dst, int32_t dst_on_device, int32_t reset) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (!dst) return fail(h, CORR_E_INVALID_ARG, "dst is NULL");
    if (dst_on_device && !aligned(dst, 8)) return fail(h, CORR_E_INVALID_ARG, "dst must be 8-byte aligned");
    const size_t bytes = (size_t)corr_visibility_bytes(&h->p);
    hipError_t e;
    if (h->zflag) {
        // batch member: whether the accumulators are logically zero is the
        // device flag's to say (graph replays do not pass through the host)
        void *target = dst;
        if (!dst_on_device) {
            if (!h->dump_tmp && (e = hipMalloc(&h->dump_tmp, bytes)) != hipSuccess)
                return hip_fail(h, e, "hipMalloc dump staging");
            target = h->dump_tmp;
        }
        if (default_dump(&h->p) && aligned(target, 16))
            e = launch_dump_copy(h->acc, target, (int64_t)(bytes / 4), h->zflag, h->stream);
        else
            e = launch_dump_convert(h->C, h->N, h->p.layout, h->p.order, h->prec == P_INT8 ? 1 : 0, h->acc, target,
                                    h->stream, h->zflag);
        if (e != hipSuccess) return hip_fail(h, e, "dump launch");
        if (reset && (e = launch_set_flag(h->zflag, 1, h->stream)) != hipSuccess) return hip_fail(h, e, "flag launch");
        if (!dst_on_device) {
            if ((e = hipMemcpyAsync(dst, target, bytes, hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
                return hip_fail(h, e, "hipMemcpyAsync dump");
            if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
        }
        if (reset) h->n_integrated = 0;
        h->err.clear();
        return CORR_OK;
    }
    if (h->acc_zero) {
        if (dst_on_device) {
            e = launch_zero(dst, (int64_t)(bytes / 4), h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "zero launch");
        } else {
            e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
            std::memset(dst, 0, bytes);
        }
    } else if (default_dump(&h->p)) {
        e = hipMemcpyAsync(dst, h->acc, bytes, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "hipMemcpyAsync dump");
        if (!dst_on_device && (e = hipStreamSynchronize(h->stream)) != hipSuccess)
            return hip_fail(h, e, "hipStreamSynchronize");
    } else {
        void *target = dst;
        if (!dst_on_device) {
            if (!h->dump_tmp && (e = hipMalloc(&h->dump_tmp, bytes)) != hipSuccess)
                return hip_fail(h, e, "hipMalloc dump staging");
            target = h->dump_tmp;
        }
        e = launch_dump_convert(h->C, h->N, h->p.layout, h->p.order, h->prec == P_INT8 ? 1 : 0, h->acc, target,
                                h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "dump convert launch");
        if (!dst_on_device) {
            if ((e = hipMemcpyAsync(dst, target, bytes, hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
                return hip_fail(h, e, "hipMemcpyAsync dump");
            if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
        }
    }
    if (reset) {
        h->acc_zero = true;
        h->n_integrated = 0;
    }
    h->err.clear();
    return CORR_OK;
}

corr_status corr_copy_spectra(corr_handle h, void *dst, int32_t dst_on_device) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (!dst) return fail(h, CORR_E_INVALID_ARG, "dst is NULL");
    if (h->n_held == 0) return fail(h, CORR_E_STATE, "no spectra held");
    const size_t bytes = (size_t)corr_spectra_bytes(&h->p, h->n_held);
    hipError_t e;
    void *target = dst;
    void *tmp = nullptr;
    if (!dst_on_device) {
        if ((e = hipMalloc(&tmp, bytes)) != hipSuccess) return hip_fail(h, e, "hipMalloc spectra staging");
        target = tmp;
    }
    e = launch_export(h->prec, h->C, h->N, h->n_held, h->lay, h->spec, target, h->stream);
    if (e == hipSuccess && !dst_on_device) {
        e = hipMemcpyAsync(dst, tmp, bytes, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(h, e, "copy spectra");
    h->err.clear();
    return CORR_OK;
}

corr_status corr_get_counts(corr_handle h, int32_t *n_held, int64_t *n_integrated) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (!n_held || !n_integrated) return fail(h, CORR_E_INVALID_ARG, "output pointer is NULL");
    *n_held = h->n_held;
    *n_integrated = h->n_integrated;
    return CORR_OK;
}


corr_status corr_set_tile(corr_handle h, int32_t tile) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (tile != 0 && tile != 64 && tile != 128) return fail(h, CORR_E_INVALID_ARG, "tile must be 0, 64 or 128");
    h->tile = tile;
    return CORR_OK;
}

corr_status corr_autotune(corr_handle h, int32_t n_spectra, int32_t *tile_out) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (n_spectra < 1) return fail(h, CORR_E_INVALID_ARG, "n_spectra must be >= 1");
    if (h->n_held == 0 || n_spectra > h->n_held) return fail(h, CORR_E_STATE, "autotune needs held spectra");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(h->stream, &cs);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) return fail(h, CORR_E_STATE, "cannot autotune while capturing");
    const int n_tb = (n_spectra + h->TB - 1) / h->TB;
    const TuneKey key{h->arch, 0, h->prec, (h->N + 63) / 64, h->C, n_tb, h->tb_major ? 1 : 0};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            h->tile = it->second.tile;
            if (tile_out) *tile_out = h->tile;
            return CORR_OK;
        }
    }
    const int Ct = tune_channels(h);
    const int cand[2] = {64, 128};
    const int def_tile = (h->N <= 64 || h->prec == P_FP32) ? 64 : 128;
    float best_ms = 0, def_ms = 0;
    int best = 0;
    {
        TuneScope sc;
        if ((e = sc.create(2, (size_t)Ct * h->B * 8)) != hipSuccess) return hip_fail(h, e, "autotune setup");
        void *tmp = sc.tmp;
        for (int c : cand) {
            float ms = 0;
            e = launch_xengine(h->prec, c, Ct, h->N, n_spectra, h->spec, h->lay, x_scale(h), tmp, tmp, 1, h->stream);
            for (int r = 0; e == hipSuccess && r < 3; ++r) {
                e = hipEventRecord(sc.ev[0], h->stream);
                if (e == hipSuccess)
                    e = launch_xengine(h->prec, c, Ct, h->N, n_spectra, h->spec, h->lay, x_scale(h), tmp, tmp, 1,
                                       h->stream);
                if (e == hipSuccess) e = hipEventRecord(sc.ev[1], h->stream);
                if (e == hipSuccess) e = hipEventSynchronize(sc.ev[1]);
                float t = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&t, sc.ev[0], sc.ev[1]);
                ms = (r == 0 || t < ms) ? t : ms;
            }
            if (e != hipSuccess) break;
            if (c == def_tile) def_ms = ms;
            if (!best || ms < best_ms) {
                best = c;
                best_ms = ms;
            }
        }
    }
    if (e != hipSuccess) return hip_fail(h, e, "autotune");
    if (best_ms > kTuneMargin * def_ms) best = def_tile;    // within the timing noise: keep the built-in
    h->tile = best;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_store_locked(key, {best, h->tb_major ? 1 : 0});
    }
    if (tile_out) *tile_out = best;
    h->err.clear();
    return CORR_OK;
}

corr_status corr_set_spectra_layout(corr_handle h, int32_t time_block_major) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (time_block_major < -1 || time_block_major > 1)
        return fail(h, CORR_E_INVALID_ARG, "time_block_major must be -1, 0 or 1");
    if (h->batch_member) return fail(h, CORR_E_STATE, "the batch plan holds its sub-arrays' layouts");
    const bool tb = time_block_major < 0 ? default_tb_major(h->C, h->N, elem_bytes(h->prec)) : time_block_major == 1;
    if (tb != h->tb_major) {
        h->tb_major = tb;
        h->lay = spec_layout_of(h->C, h->N, h->n_tb_cap, tb);
        h->n_held = 0;                                   // the held spectra were in the other order
        h->held_from_fengine = false;
    }
    h->err.clear();
    return CORR_OK;
}

corr_status corr_autotune_fx(corr_handle h, const void *d_volts, int64_t ld_samples, int32_t n_spectra,
                             const float *d_inv_scale, corr_tuning *out) {
    if (!h) return fail(nullptr, CORR_E_INVALID_ARG, "handle is NULL");
    if (!d_volts || !aligned(d_volts, 8)) return fail(h, CORR_E_INVALID_ARG, "d_volts must be 8-byte aligned");
    if (d_inv_scale && !aligned(d_inv_scale, 4)) return fail(h, CORR_E_INVALID_ARG, "d_inv_scale misaligned");
    if (n_spectra < 1 || n_spectra > h->p.n_integrate)
        return fail(h, CORR_E_INVALID_ARG, "need 1 <= n_spectra <= n_integrate");
    if (ld_samples < (int64_t)n_spectra * h->C)
        return fail(h, CORR_E_INVALID_ARG, "ld_samples < n_spectra * n_channels");
    if (h->prec == P_INT8 && !d_inv_scale) return fail(h, CORR_E_INVALID_ARG, "int8 needs a per-channel scale");
    if (h->batch_member) return fail(h, CORR_E_STATE, "the batch plan holds its sub-arrays' layouts");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(h->stream, &cs);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) return fail(h, CORR_E_STATE, "cannot autotune while capturing");

    const int n_tb = (n_spectra + h->TB - 1) / h->TB;
    const bool def_tb = default_tb_major(h->C, h->N, elem_bytes(h->prec));
    const int def_tile = (h->N <= 64 || h->prec == P_FP32) ? 64 : 128;
    const TuneKey key{h->arch, 1, h->prec, (h->N + 63) / 64, h->C, n_tb, 0};
    TuneVal best{def_tile, def_tb ? 1 : 0};
    float best_ms = 0, def_ms = 0;
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            best = it->second;
            cached = true;
        }
    }
    const float *inv = d_inv_scale ? d_inv_scale : h->unit_scale;
    const float2 *v = static_cast<const float2 *>(d_volts);
    h->n_held = 0;                                        // the spectra buffer is overwritten from here on
    h->held_from_fengine = false;
    if ((e = launch_scale2(h->C, d_inv_scale, h->scale2, h->stream)) != hipSuccess) return hip_fail(h, e, "scale2");
    if (!cached) {
        // F-engine on every channel, X-engine on some of them into scratch
        // accumulators (the integration is untouched), scaled up to C
        const int Ct = tune_channels(h);
        TuneScope sc;
        if ((e = sc.create(3, (size_t)Ct * h->B * 8)) != hipSuccess) return hip_fail(h, e, "autotune setup");
        void *tmp = sc.tmp;
        hipEvent_t *ev = sc.ev;
        best_ms = 0;
        bool first = true;
        for (int o = 0; o < 2 && e == hipSuccess; ++o) {
            const bool tb = o == 0 ? def_tb : !def_tb;
            const SpecLayout lay = spec_layout_of(h->C, h->N, h->n_tb_cap, tb);
            for (int tile : {64, 128}) {
                float ms = 0;
                for (int r = 0; e == hipSuccess && r < 3; ++r) {
                    e = hipEventRecord(ev[0], h->stream);
                    if (e == hipSuccess)
                        e = launch_fengine(h->prec, h->C, h->N, v, ld_samples, n_spectra, inv, h->twiddle, h->spec,
                                           lay, FScratch{h->gscr, h->gscr_bytes}, 0, h->stream);
                    if (e == hipSuccess) e = hipEventRecord(ev[1], h->stream);
                    if (e == hipSuccess)
                        e = launch_xengine(h->prec, tile, Ct, h->N, n_spectra, h->spec, lay,
                                           h->prec == P_INT8 ? nullptr : h->scale2, tmp, tmp, 1, h->stream);
                    if (e == hipSuccess) e = hipEventRecord(ev[2], h->stream);
                    if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
                    float tf = 0, tx = 0;
                    if (e == hipSuccess) e = hipEventElapsedTime(&tf, ev[0], ev[1]);
                    if (e == hipSuccess) e = hipEventElapsedTime(&tx, ev[1], ev[2]);
                    const float t = tf + tx * (float)h->C / (float)Ct;
                    if (r > 0) ms = (r == 1 || t < ms) ? t : ms;           // the first run warms up
                }
                if (e != hipSuccess) break;
                if (tb == def_tb && tile == def_tile) def_ms = ms;
                if (first || ms < best_ms) {
                    best = {tile, tb ? 1 : 0};
                    best_ms = ms;
                    first = false;
                }
            }
        }
        if (e != hipSuccess) return hip_fail(h, e, "autotune");
        if (best_ms > kTuneMargin * def_ms) {                // within the timing noise: keep the built-in
            best = {def_tile, def_tb ? 1 : 0};
            best_ms = def_ms;
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_store_locked(key, best);
    }
    // keep the choice and leave the handle holding these spectra in its order
    h->tile = best.tile;
    h->tb_major = best.tb_major == 1;
    h->lay = spec_layout_of(h->C, h->N, h->n_tb_cap, h->tb_major);
    e = launch_fengine(h->prec, h->C, h->N, v, ld_samples, n_spectra, inv, h->twiddle, h->spec, h->lay,
                       FScratch{h->gscr, h->gscr_bytes}, 0, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "fengine launch");
    h->n_held = n_spectra;
    h->held_from_fengine = true;
    if (out) {
        out->tile = best.tile;
        out->time_block_major = best.tb_major;
        out->default_tile = def_tile;
        out->default_time_block_major = def_tb ? 1 : 0;
        out->ms_default = cached ? -1.0f : def_ms;
        out->ms_tuned = cached ? -1.0f : best_ms;
    }
    h->err.clear();
    return CORR_OK;
}

// Bytes of a batch work plan for n sub-arrays: two group headers, then the
// descriptors of both groups.
static_assert(sizeof(XQueue) % alignof(XDesc) == 0, "descriptors follow the two headers");
static size_t plan_size(int n) { return 2 * sizeof(XQueue) + (size_t)n * sizeof(XDesc); }

static void destroy_batch(corr_batch *b) {
    if (b->stream || !b->subs.empty()) (void)hipStreamSynchronize(b->stream);
    for (corr_ctx *h : b->subs) destroy_ctx(h);
    (void)hipFree(b->d_plan);
    (void)hipFree(b->d_counter);
    (void)hipFree(b->d_zflag);
    (void)hipFree(b->d_gscr);
    if (b->h_plan) (void)hipHostFree(b->h_plan);
    delete b;
}

corr_status corr_create_batched(const corr_params *params, int32_t n, void *hip_stream, corr_batch_handle *out) {
    if (!params || !out) return fail(nullptr, CORR_E_INVALID_ARG, "params and out must not be NULL");
    if (n < 1 || n > 65536) return fail(nullptr, CORR_E_INVALID_ARG, "n must be in 1..65536");
    std::string msg;
    uint64_t need = 0;
    int64_t gscr_bytes = 0;                  // one scratch for all: the largest any sub-array needs
    for (int i = 0; i < n; ++i) {
        corr_status s = check_params(&params[i], msg);
        if (s != CORR_OK) return fail(nullptr, s, "sub-array " + std::to_string(i) + ": " + msg);
        if (params[i].precision != params[0].precision)
            return fail(nullptr, CORR_E_UNSUPPORTED, "all sub-arrays must share one precision");
        const int64_t N = n_inputs(&params[i]);
        const int TB = time_block(params[i].precision);
        need += (uint64_t)spec_buffer_bytes(params[i].n_channels, (int)N, (params[i].n_integrate + TB - 1) / TB,
                                            elem_bytes(params[i].precision)) +
                (uint64_t)params[i].n_channels * (N * (N + 1) / 2) * 8;
        gscr_bytes = std::max(gscr_bytes, gather_scratch_bytes(params[i].n_channels, (int)N,
                                                               (params[i].n_integrate + TB - 1) / TB));
    }
    need += (uint64_t)gscr_bytes;
    if (params[0].device_mem_cap && need > params[0].device_mem_cap)
        return fail(nullptr, CORR_E_NOMEM, "batch needs " + std::to_string(need) + " bytes, over the cap");
    corr_batch *b = new (std::nothrow) corr_batch();
    if (!b) return fail(nullptr, CORR_E_NOMEM, "host allocation failed");
    b->prec = params[0].precision;
    b->stream = static_cast<hipStream_t>(hip_stream);
    for (int i = 0; i < n; ++i) {
        corr_params p = params[i];
        p.device_mem_cap = 0;
        corr_handle h = nullptr;
        g_no_own_scratch = true;
        corr_status s = corr_create(&p, hip_stream, &h);
        g_no_own_scratch = false;
        if (s != CORR_OK) {
            std::string m = "sub-array " + std::to_string(i) + ": " + g_err;
            destroy_batch(b);
            return fail(nullptr, s, m);
        }
        h->batch_member = true;
        h->acc_zero = false;                     // the device flag decides
        b->subs.push_back(h);
    }
    // every sub-array starts logically zero: its flag is set, its
    // accumulators are never cleared in memory
    hipError_t ez = hipMalloc(&b->d_zflag, (size_t)n * sizeof(int));
    if (ez == hipSuccess)
        ez = hipMemcpy(b->d_zflag, std::vector<int>(n, 1).data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice);
    if (ez != hipSuccess) {
        destroy_batch(b);
        return fail(nullptr, CORR_E_HIP, std::string("batch flags: ") + hipGetErrorString(ez));
    }
    for (int i = 0; i < n; ++i) b->subs[i]->zflag = b->d_zflag + i;
    if (gscr_bytes && (ez = hipMalloc(&b->d_gscr, (size_t)gscr_bytes)) != hipSuccess) {
        destroy_batch(b);
        return fail(nullptr, ez == hipErrorOutOfMemory ? CORR_E_NOMEM : CORR_E_HIP,
                    std::string("batch F-engine scratch: ") + hipGetErrorString(ez));
    }
    for (corr_ctx *h : b->subs) {
        h->owns_gscr = false;
        if (gather_scratch_bytes(h->C, h->N, h->n_tb_cap)) {
            h->gscr = b->d_gscr;
            h->gscr_bytes = gscr_bytes;
        }
    }
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const size_t plan_bytes = plan_size(n);
    if (e == hipSuccess) e = hipMalloc(&b->d_plan, plan_bytes);
    if (e == hipSuccess) e = hipMalloc(&b->d_counter, 2 * kXcds * kCounterStride * sizeof(unsigned int));
    if (e == hipSuccess) e = hipHostMalloc(&b->h_plan, plan_bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        destroy_batch(b);
        return fail(nullptr, CORR_E_HIP, std::string("batch setup: ") + hipGetErrorString(e));
    }
    b->num_cus = cus > 0 ? cus : 256;
    *out = b;
    return CORR_OK;
}

corr_status corr_batch_get(corr_batch_handle b, int32_t i, corr_handle *h) {
    if (!b || !h) return fail(nullptr, CORR_E_INVALID_ARG, "batch and h must not be NULL");
    if (i < 0 || i >= (int)b->subs.size()) return fail(nullptr, CORR_E_INVALID_ARG, "sub-array index out of range");
    *h = b->subs[i];
    return CORR_OK;
}

corr_status corr_xengine_batched(corr_batch_handle b, const int32_t *n_spectra) {
    if (!b || !n_spectra) return fail(nullptr, CORR_E_INVALID_ARG, "batch and n_spectra must not be NULL");
    const int n = (int)b->subs.size();
    for (int i = 0; i < n; ++i) {
        corr_ctx *h = b->subs[i];
        const int ns = n_spectra[i];
        if (ns < 0) return fail(nullptr, CORR_E_INVALID_ARG, "n_spectra must be >= 0");
        if (ns == 0) continue;
        if (h->n_held == 0 || ns > h->n_held)
            return fail(nullptr, CORR_E_STATE, "sub-array " + std::to_string(i) + ": n_spectra exceeds held");
        if (h->prec == P_INT8 && h->n_integrated + ns > CORR_INT8_MAX_INTEGRATE)
            return fail(nullptr, CORR_E_OVERFLOW, "sub-array " + std::to_string(i) + ": int8 integration too long");
    }
    // A sub-array with at least kDirectWaves work items per resident
    // workgroup of its block size fills the GPU on its own: it runs as an
    // ordinary X-engine launch.  Measured on the 64-sub-array FP16 batch: the
    // 42 such sub-arrays took 100.7 ms in the persistent launches against
    // 96.6 ms as their own launches (the persistent kernel's unbroken load
    // runs at a lower clock), the other 22 took 2.08 against 2.23 ms.
    constexpr int kDirectWaves = 4;
    std::vector<int> direct;
    // descriptors in two groups (64- then 128-input blocks), each largest item
    // first; XCD x's queue of a group takes channels [x C/8, (x+1) C/8) of each
    // of its sub-arrays in that order
    std::vector<std::pair<int64_t, int>> order[2];
    for (int i = 0; i < n; ++i) {
        if (!n_spectra[i]) continue;
        const corr_ctx *h = b->subs[i];
        const int t = effective_tile(h);
        const int64_t nb = (h->N + t - 1) / t;
        const int64_t items = (int64_t)h->C * (nb * (nb + 1) / 2);
        const int64_t resident = (int64_t)b->num_cus * (t == 64 ? 4 : 2);
        if (items >= kDirectWaves * resident) {
            direct.push_back(i);
            continue;
        }
        const int64_t n_tb = (n_spectra[i] + h->TB - 1) / h->TB;
        order[t == 64 ? 0 : 1].push_back({n_tb * t * t, i});
    }
    hipError_t e;
    for (int i : direct) {
        corr_ctx *h = b->subs[i];
        e = launch_xengine(h->prec, effective_tile(h), h->C, h->N, n_spectra[i], h->spec, h->lay, x_scale(h), h->acc,
                           h->acc, 0, b->stream, h->zflag);
        if (e == hipSuccess) e = launch_set_flag(h->zflag, 0, b->stream);
        if (e != hipSuccess) return fail(nullptr, CORR_E_HIP, std::string("direct launch: ") + hipGetErrorString(e));
        h->n_integrated += n_spectra[i];
        h->acc_zero = false;
    }
    if (order[0].empty() && order[1].empty()) return CORR_OK;
    XQueue q[2] = {};
    std::vector<XDesc> d;
    for (int g = 0; g < 2; ++g) {
        std::stable_sort(order[g].begin(), order[g].end(),
                         [](const auto &x, const auto &y) { return x.first > y.first; });
        q[g].n_desc = (int)order[g].size();
        q[g].desc_offset = (int)d.size();
        for (const auto &o : order[g]) {
            const corr_ctx *h = b->subs[o.second];
            const int ns = n_spectra[o.second];
            XDesc x{};
            x.spec = static_cast<const uint8_t *>(h->spec);
            x.acc = h->acc;
            x.scale2 = x_scale(h);
            x.k_stride = h->lay.ks;
            x.tb_stride = h->lay.ts;
            x.B = h->B;
            x.C = h->C;
            x.N = h->N;
            x.n_tb = (ns + h->TB - 1) / h->TB;
            x.tv = ns - (x.n_tb - 1) * h->TB;
            x.tile = effective_tile(h);
            const int nb = (h->N + x.tile - 1) / x.tile;
            x.n_tiles = nb * (nb + 1) / 2;
            x.first_call = 0;
            x.zflag = h->zflag;               // set: write instead of add (cleared after the launch)
            for (int xc = 0; xc < kXcds; ++xc) {
                x.qbegin[xc] = q[g].qlen[xc];
                const int c_lo = xc * h->C / kXcds, c_hi = (xc + 1) * h->C / kXcds;
                q[g].qlen[xc] += (int64_t)(c_hi - c_lo) * x.n_tiles;
            }
            d.push_back(x);
        }
        for (int xc = 0; xc < kXcds; ++xc)
            if (q[g].qlen[xc] >= ((int64_t)1 << 31))
                return fail(nullptr, CORR_E_UNSUPPORTED, "more than 2^31 work items on one XCD");
    }
    const size_t bytes = plan_size((int)d.size());
    std::vector<uint8_t> plan(bytes);
    std::memcpy(plan.data(), q, sizeof(q));
    std::memcpy(plan.data() + sizeof(q), d.data(), d.size() * sizeof(XDesc));
    if (plan != b->last) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if ((e = hipStreamIsCapturing(b->stream, &cs)) != hipSuccess)
            return fail(nullptr, CORR_E_HIP, std::string("hipStreamIsCapturing: ") + hipGetErrorString(e));
        if (cs != hipStreamCaptureStatusNone)
            return fail(nullptr, CORR_E_STATE, "the work list changed during graph capture; call once before capturing");
        // the previous upload may still be reading the pinned staging buffer
        if ((e = hipStreamSynchronize(b->stream)) != hipSuccess)
            return fail(nullptr, CORR_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
        std::memcpy(b->h_plan, plan.data(), bytes);
        if ((e = hipMemcpyAsync(b->d_plan, b->h_plan, bytes, hipMemcpyHostToDevice, b->stream)) != hipSuccess)
            return fail(nullptr, CORR_E_HIP, std::string("plan upload: ") + hipGetErrorString(e));
        b->last.swap(plan);
    }
    const int groups = (q[0].n_desc ? 1 : 0) | (q[1].n_desc ? 2 : 0);
    e = launch_xengine_batched(b->prec, reinterpret_cast<const XQueue *>(b->d_plan),
                               reinterpret_cast<const XDesc *>(b->d_plan + 2 * sizeof(XQueue)), groups,
                               b->d_counter, b->num_cus, b->stream);
    if (e != hipSuccess) return fail(nullptr, CORR_E_HIP, std::string("batched launch: ") + hipGetErrorString(e));
    for (const auto &grp : order)
        for (const auto &o : grp) {
            b->subs[o.second]->n_integrated += n_spectra[o.second];
            b->subs[o.second]->acc_zero = false;
        }
    return CORR_OK;
}

corr_status corr_destroy_batched(corr_batch_handle b) {
    if (!b) return fail(nullptr, CORR_E_INVALID_ARG, "batch is NULL");
    destroy_batch(b);
    return CORR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// X-engine without allocation.  The staging of caller spectra in the
// X-engine's held-row layout (the handle's spectra buffer in corr_xengine)
// is a file-scope device array instead, kNoAllocScratch bytes per device:
// the per-channel scales s_k^2 first, then the held rows of as many
// channels as fit, correlated chunk by chunk.  Every call on a device shares
// its array; calls that overlap on one device race.
namespace {

constexpr int64_t kNoAllocScratch = (int64_t)32 << 20;
constexpr int kNoAllocMaxDevices = 64;

}  // namespace

static __device__ __align__(256) uint8_t scratch[kNoAllocScratch];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocMaxDevices] = {};

// The device address of `scratch` on the current device (taken once per
// device); the array's name is only a host-side stand-in.
hipError_t scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

corr_status corr_xengine_noalloc(const corr_params *params, const void *d_spectra, int32_t n_spectra,
                                 const float *d_inv_scale, void *d_vis, int32_t accumulate, void *hip_stream) {
    std::string msg;
    corr_status s = check_params(params, msg);
    if (s != CORR_OK) return fail(nullptr, s, msg);
    if (!default_dump(params))
        return fail(nullptr, CORR_E_UNSUPPORTED, "the no-alloc X-engine writes the lower-triangle, channel-major layout");
    if (n_spectra < 1) return fail(nullptr, CORR_E_INVALID_ARG, "n_spectra must be >= 1");
    if (!d_spectra || !aligned(d_spectra, 16))
        return fail(nullptr, CORR_E_INVALID_ARG, "d_spectra must be a 16-byte aligned device pointer");
    if (!d_vis || !aligned(d_vis, 8)) return fail(nullptr, CORR_E_INVALID_ARG, "d_vis must be an 8-byte aligned device pointer");
    if (accumulate != 0 && accumulate != 1) return fail(nullptr, CORR_E_INVALID_ARG, "accumulate must be 0 or 1");
    const int prec = params->precision;
    if (d_inv_scale && (prec == P_FP32 || prec == P_INT8))
        return fail(nullptr, CORR_E_INVALID_ARG, "d_inv_scale applies only to FP16/FP8 spectra");
    if (d_inv_scale && !aligned(d_inv_scale, 4)) return fail(nullptr, CORR_E_INVALID_ARG, "d_inv_scale misaligned");
    if (prec == P_INT8 && n_spectra > CORR_INT8_MAX_INTEGRATE)
        return fail(nullptr, CORR_E_OVERFLOW, "int8 call over 66572 spectra could overflow int32");
    const int N = (int)n_inputs(params), C = params->n_channels;
    const int TB = time_block(prec);
    const int n_tb = (n_spectra + TB - 1) / TB;
    // scratch: s_k^2 (C floats, rounded up to 256 bytes), then channel-major
    // held rows of nk channels
    const int64_t s2_bytes = ((int64_t)C * 4 + 255) / 256 * 256;
    const SpecLayout lay{(int64_t)n_tb * N * 2 * kRowBytes + kChannelPad, (int64_t)N * 2 * kRowBytes};
    const int64_t nk64 = (kNoAllocScratch - s2_bytes) / lay.ks;
    if (nk64 < 1) {
        char b[200];
        snprintf(b, sizeof b, "one channel of %d inputs x %d spectra needs %lld scratch bytes; the no-alloc "
                 "scratch holds %lld", N, n_spectra, (long long)(s2_bytes + lay.ks), (long long)kNoAllocScratch);
        return fail(nullptr, CORR_E_UNSUPPORTED, b);
    }
    const int nk = (int)std::min<int64_t>(nk64, C);

    // ---- HIP from here on ----
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    void *base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
    float *s2 = static_cast<float *>(base);
    uint8_t *spec = static_cast<uint8_t *>(base) + s2_bytes;
    const bool scaled = prec == P_FP16 || prec == P_FP8;
    if (scaled && (e = launch_scale2(C, d_inv_scale, s2, stream)) != hipSuccess)
        return hip_fail(nullptr, e, "scale2 launch");
    const int tile = (N <= 64 || prec == P_FP32) ? 64 : 128;
    const int64_t B = (int64_t)N * (N + 1) / 2;
    for (int k0 = 0; k0 < C; k0 += nk) {
        const int n = std::min(nk, C - k0);
        e = launch_ingest_channels(prec, C, k0, n, N, n_spectra, lay, d_spectra, spec, stream);
        if (e != hipSuccess) return hip_fail(nullptr, e, "ingest launch");
        uint8_t *vis = static_cast<uint8_t *>(d_vis) + (int64_t)k0 * B * 8;
        e = launch_xengine(prec, tile, n, N, n_spectra, spec, lay, scaled ? s2 + k0 : nullptr, vis, vis,
                           accumulate ? 0 : 1, stream);
        if (e != hipSuccess) return hip_fail(nullptr, e, "xengine launch");
    }
    return CORR_OK;
}

}  // extern "C"
