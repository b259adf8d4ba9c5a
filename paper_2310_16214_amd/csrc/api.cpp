// Exported C entry points of libppx.so: argument validation (before any HIP
// runtime call), configuration resolution and kernel dispatch, plus the
// per-device state (limits, twiddle table) and thread-local error messages.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ppx_internal.h"

namespace ppx {

// ------------------------------------------------------------------ errors
static thread_local std::string t_err;

int fail(int code, const std::string &msg) {
    t_err = msg;
    return code;
}

int fail_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return PPX_OK;
    t_err = std::string(what) + ": " + hipGetErrorString(e);
    return PPX_EHIP;
}

// ------------------------------------------------------------ device state
// The FFT twiddle tables live in static device arrays, filled once per device
// when it is first used: setting a device up allocates no device memory.
// w[m] = exp(-2 pi i m / 2^14); the large-N tables w_{2^23}^j (j < 1024) and
// w_{2^13}^j (j < 1024) followed by w_8^j (j < 8).
static __device__ float2 g_tw_small[1 << kFftLog2NMax];
static __device__ float2 g_tw_large_lo[1024];
static __device__ float2 g_tw_large_hi[1024 + 8];

namespace {
std::mutex g_dev_mu;
// host images of the tables (filled under g_dev_mu)
float g_tw_host[2 << kFftLog2NMax];
float g_tw_lo_host[2 * 1024];
float g_tw_hi_host[2 * (1024 + 8)];
std::vector<DeviceInfo *> g_devices;  // indexed by device ordinal; never freed
bool g_any_device = false;
int64_t g_lds_limit = kStaticLdsPerBlock;
}  // namespace

int current_device_or_zero() {
    if (!g_any_device) return 0;
    int d = 0;
    return hipGetDevice(&d) == hipSuccess ? d : 0;
}

int64_t lds_limit() { return g_lds_limit; }

const DeviceInfo *device_info_if_ready() {
    if (!g_any_device) return nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    return dev < (int)g_devices.size() ? g_devices[dev] : nullptr;
}

const DeviceInfo *device_info() {
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        fail(PPX_EDEVICE, std::string("no HIP device available: ") + hipGetErrorString(e));
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (dev < (int)g_devices.size() && g_devices[dev]) return g_devices[dev];
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        fail(PPX_EDEVICE, "hipGetDeviceProperties failed");
        return nullptr;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        fail(PPX_EDEVICE, std::string("libppx is built for gfx950; device is ") + prop.gcnArchName);
        return nullptr;
    }
    auto *di = new DeviceInfo();
    di->device = dev;
    di->cus = prop.multiProcessorCount;
    di->lds_per_block = (int64_t)prop.sharedMemPerBlock;
    di->lds_per_cu = (int64_t)prop.maxSharedMemoryPerMultiProcessor;
    di->max_threads_per_cu = prop.maxThreadsPerMultiProcessor;
    di->clock_khz = prop.clockRate;
    di->l2_bytes = prop.l2CacheSize;
    di->arch = prop.gcnArchName;
    // Twiddle tables: the largest supported FFT's (every smaller size indexes
    // it with a stride) and the large-N tables, copied into this device's
    // static arrays.
    fft_host_twiddles(g_tw_host);
    fft_large_host_twiddles(g_tw_lo_host, g_tw_hi_host);
    void *dtw = nullptr, *dlo = nullptr, *dhi = nullptr;
    if (hipGetSymbolAddress(&dtw, HIP_SYMBOL(g_tw_small)) != hipSuccess ||
        hipGetSymbolAddress(&dlo, HIP_SYMBOL(g_tw_large_lo)) != hipSuccess ||
        hipGetSymbolAddress(&dhi, HIP_SYMBOL(g_tw_large_hi)) != hipSuccess ||
        hipMemcpy(dtw, g_tw_host, sizeof g_tw_host, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dlo, g_tw_lo_host, sizeof g_tw_lo_host, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dhi, g_tw_hi_host, sizeof g_tw_hi_host, hipMemcpyHostToDevice) != hipSuccess) {
        fail(PPX_EDEVICE, "could not set up the FFT twiddle tables");
        delete di;
        return nullptr;
    }
    di->twiddles = dtw;
    di->twiddles_large_lo = dlo;
    di->twiddles_large_hi = dhi;
    if ((int)g_devices.size() <= dev) g_devices.resize(dev + 1, nullptr);
    g_devices[dev] = di;
    g_any_device = true;
    g_lds_limit = di->lds_per_block;
    return di;
}

// ----------------------------------------------------------- validation
static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

static bool overlap_partial(const void *a, const void *b, int64_t bytes) {
    const auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    if (x == y) return false;
    return x < y + (uintptr_t)bytes && y < x + (uintptr_t)bytes;
}

static int check_shape(int64_t n, int64_t batch, int64_t elem_bytes) {
    if (!is_pow2(n) || n < PPX_MIN_N || n > PPX_MAX_N)
        return fail(PPX_EINVAL, "n must be a power of two in [16, 16384]");
    if (batch < 1) return fail(PPX_EINVAL, "batch must be >= 1");
    if (batch > (int64_t(1) << 40) / n || batch * n > INT64_MAX / elem_bytes)
        return fail(PPX_EINVAL, "batch * n is too large");
    return PPX_OK;
}

static int resolve(int op, int dtype, int64_t n, int64_t batch, const ppx_config *cfg,
                   ppx_config &c) {
    if (cfg) {
        c = *cfg;
        complete_config(op, dtype, n, c);
        return validate_config(op, dtype, n, c);
    }
    if (cached_config(op, dtype, n, c)) return PPX_OK;
    return analytical_config(op, dtype, n, batch, c);
}

}  // namespace ppx

using namespace ppx;

extern "C" {

const char *ppx_last_error(void) { return t_err.c_str(); }

int fft_batched(const void *in, void *out, int64_t n, int64_t batch, int direction,
                const ppx_config *cfg, void *stream) {
    t_err.clear();
    if (is_pow2(n) && n > PPX_MAX_N && n <= PPX_MAX_N_LARGE) {
        if (cfg) return fail(PPX_EINVAL, "n > 16384 takes a plan (fft_batched_large), not a ppx_config");
        return fft_batched_large(in, out, n, batch, direction, nullptr, stream);
    }
    if (!in || !out) return fail(PPX_EINVAL, "null pointer");
    if (!aligned16(in) || !aligned16(out)) return fail(PPX_EINVAL, "pointers must be 16-byte aligned");
    if (direction != -1 && direction != 1) return fail(PPX_EINVAL, "direction must be -1 or +1");
    int rc = check_shape(n, batch, 8);
    if (rc) return rc;
    if (overlap_partial(in, out, batch * n * 8)) return fail(PPX_EINVAL, "in and out overlap partially");
    ppx_config c;
    if ((rc = resolve(PPX_OP_FFT, PPX_C64, n, batch, cfg, c))) return rc;
    if ((batch + c.problems_per_block - 1) / c.problems_per_block > INT32_MAX)
        return fail(PPX_EINVAL, "too many workgroups");
    return launch_fft(in, out, ilog2(n), batch, c, direction == 1, static_cast<hipStream_t>(stream));
}

int fft_batched_large(const void *in, void *out, int64_t n, int64_t batch, int direction,
                      const ppx_fft_plan *plan, void *stream) {
    t_err.clear();
    if (!in || !out) return fail(PPX_EINVAL, "null pointer");
    if (!aligned16(in) || !aligned16(out)) return fail(PPX_EINVAL, "pointers must be 16-byte aligned");
    if (direction != -1 && direction != 1) return fail(PPX_EINVAL, "direction must be -1 or +1");
    if (!is_pow2(n) || n <= PPX_MAX_N || n > PPX_MAX_N_LARGE)
        return fail(PPX_EINVAL, "large FFT: n must be a power of two in (16384, 8388608]");
    if (batch < 1) return fail(PPX_EINVAL, "batch must be >= 1");
    if (batch > (int64_t(1) << 40) / n) return fail(PPX_EINVAL, "batch * n is too large");
    const int64_t bytes = batch * n * 8;
    const char *pi = static_cast<const char *>(in), *po = static_cast<const char *>(out);
    if (pi < po + bytes && po < pi + bytes)
        return fail(PPX_EINVAL, "large FFT: in and out must not overlap (out holds the intermediate)");
    ppx_fft_plan p;
    if (plan) p = *plan;
    else if (!fft_tuned_plan(n, p)) fft_default_plan(n, p);
    int rc = fft_plan_check(n, p);
    if (rc) return rc;
    if (batch * std::max<int64_t>((int64_t(1) << p.log2_n1) / p.tile_a, (n >> p.log2_n1) / p.tile_b) > INT32_MAX)
        return fail(PPX_EINVAL, "too many workgroups");
    return launch_fft_large(in, out, ilog2(n), batch, p, direction == 1, static_cast<hipStream_t>(stream));
}

int ppx_fft_plan_valid(int64_t n, const ppx_fft_plan *plan) {
    t_err.clear();
    if (!plan) return fail(PPX_EINVAL, "null plan");
    return fft_plan_check(n, *plan);
}

int ppx_enumerate_fft_plans(int64_t n, ppx_fft_plan *out, int cap) {
    t_err.clear();
    if (!is_pow2(n) || n <= PPX_MAX_N || n > PPX_MAX_N_LARGE)
        return fail(PPX_EINVAL, "large FFT: n must be a power of two in (16384, 8388608]");
    if (cap < 0 || (cap > 0 && !out)) return fail(PPX_EINVAL, "bad output buffer");
    const std::vector<ppx_fft_plan> all = fft_enumerate_plans(n);
    for (int i = 0; i < cap && i < (int)all.size(); ++i) out[i] = all[i];
    return (int)all.size();
}

int ppx_default_fft_plan(int64_t n, ppx_fft_plan *out) {
    t_err.clear();
    if (!out) return fail(PPX_EINVAL, "null plan");
    if (!is_pow2(n) || n <= PPX_MAX_N || n > PPX_MAX_N_LARGE)
        return fail(PPX_EINVAL, "large FFT: n must be a power of two in (16384, 8388608]");
    fft_default_plan(n, *out);
    return PPX_OK;
}

static int scan_common(const void *in, void *out, int64_t n, int64_t batch, int dtype,
                       const ppx_config *cfg, void *stream, bool exclusive) {
    t_err.clear();
    if (!in || !out) return fail(PPX_EINVAL, "null pointer");
    if (!aligned16(in) || !aligned16(out)) return fail(PPX_EINVAL, "pointers must be 16-byte aligned");
    if (dtype != PPX_I32 && dtype != PPX_F32 && dtype != PPX_F64)
        return fail(PPX_EINVAL, "scan dtype must be PPX_I32, PPX_F32 or PPX_F64");
    const int64_t es = dtype == PPX_F64 ? 8 : 4;
    int rc = check_shape(n, batch, es);
    if (rc) return rc;
    if (overlap_partial(in, out, batch * n * es)) return fail(PPX_EINVAL, "in and out overlap partially");
    ppx_config c;
    if ((rc = resolve(PPX_OP_SCAN, dtype, n, batch, cfg, c))) return rc;
    if ((batch + c.problems_per_block - 1) / c.problems_per_block > INT32_MAX)
        return fail(PPX_EINVAL, "too many workgroups");
    if (!device_info()) return PPX_EDEVICE;
    return launch_scan(in, out, ilog2(n), batch, dtype, c, static_cast<hipStream_t>(stream), exclusive);
}

int scan_batched(const void *in, void *out, int64_t n, int64_t batch, int dtype,
                 const ppx_config *cfg, void *stream) {
    return scan_common(in, out, n, batch, dtype, cfg, stream, false);
}

int scan_exclusive_batched(const void *in, void *out, int64_t n, int64_t batch, int dtype,
                           const ppx_config *cfg, void *stream) {
    return scan_common(in, out, n, batch, dtype, cfg, stream, true);
}

int tridiag_batched(const void *a, const void *b, const void *c, const void *d, void *x,
                    int64_t n, int64_t batch, int dtype, const ppx_config *cfg, void *stream) {
    t_err.clear();
    if (!a || !b || !c || !d || !x) return fail(PPX_EINVAL, "null pointer");
    if (!aligned16(a) || !aligned16(b) || !aligned16(c) || !aligned16(d) || !aligned16(x))
        return fail(PPX_EINVAL, "pointers must be 16-byte aligned");
    if (dtype != PPX_F32 && dtype != PPX_F64)
        return fail(PPX_EINVAL, "tridiagonal dtype must be PPX_F32 or PPX_F64");
    const int64_t es = dtype == PPX_F64 ? 8 : 4;
    int rc = check_shape(n, batch, es);
    if (rc) return rc;
    const int64_t bytes = batch * n * es;
    const void *abc[3] = {a, b, c};
    for (const void *p : abc)
        if (p == (const void *)x || overlap_partial(p, x, bytes))
            return fail(PPX_EINVAL, "x may alias d only");
    if (overlap_partial(d, x, bytes)) return fail(PPX_EINVAL, "x and d overlap partially");
    ppx_config cc;
    if ((rc = resolve(PPX_OP_TRIDIAG, dtype, n, batch, cfg, cc))) return rc;
    if ((batch + cc.problems_per_block - 1) / cc.problems_per_block > INT32_MAX)
        return fail(PPX_EINVAL, "too many workgroups");
    return launch_tridiag(a, b, c, d, x, ilog2(n), batch, dtype, cc, static_cast<hipStream_t>(stream));
}

int ppx_config_valid(int op, int dtype, int64_t n, const ppx_config *cfg) {
    t_err.clear();
    if (!cfg) return fail(PPX_EINVAL, "null config");
    ppx_config c = *cfg;
    complete_config(op, dtype, n, c);
    return validate_config(op, dtype, n, c);
}

int ppx_default_config(int op, int dtype, int64_t n, ppx_config *out) {
    t_err.clear();
    if (!out) return fail(PPX_EINVAL, "null output");
    return default_config(op, dtype, n, *out);
}

int ppx_resolve_config(int op, int dtype, int64_t n, int64_t batch, ppx_config *out) {
    t_err.clear();
    if (!out) return fail(PPX_EINVAL, "null output");
    if (batch < 1) return fail(PPX_EINVAL, "batch must be >= 1");
    return resolve(op, dtype, n, batch, nullptr, *out);
}

int ppx_enumerate_configs(int op, int dtype, int64_t n, ppx_config *out, int cap) {
    t_err.clear();
    return enumerate_configs(op, dtype, n, out, cap);
}

}  // extern "C"
