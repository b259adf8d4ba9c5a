// Internal declarations shared by the translation units of libppx.so.
// Host-side only: kernels live in fft.hip, scan.hip, tridiag.hip, fused.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ppx.h"

namespace ppx {

// ---- error reporting (thread-local message behind ppx_last_error) ----
int fail(int code, const std::string &msg);
int fail_hip(hipError_t e, const char *what);

// ---- static description of the target (gfx950) used by the validity
// predicate when no GPU is present.  The runtime limits read from the device
// replace these at first use on a GPU (see device_info()). ----
constexpr int kWave = 64;
constexpr int kMaxThreadsPerBlock = 1024;
constexpr int kMinThreadsPerBlock = 64;
constexpr int kMaxProblemsPerBlock = 64;
constexpr int kMaxElemsPerThread = 32;
// float64 scan: at most 16 values per thread (two sets of 32 do not fit the
// registers of a 1024-thread workgroup).
constexpr int kScanF64MaxElems = 16;
constexpr int64_t kStaticLdsPerBlock = 160 * 1024;  // gfx950 LDS per CU

struct DeviceInfo {
    int device = -1;
    int cus = 0;
    int64_t lds_per_block = kStaticLdsPerBlock;
    int64_t lds_per_cu = kStaticLdsPerBlock;
    int max_threads_per_cu = 2048;
    int clock_khz = 0;
    int64_t l2_bytes = 0;
    std::string arch;
    const void *twiddles = nullptr;  // device table w[m] = exp(-2 pi i m/NMAX)
    // large-N tables: w_{2^23}^j (j < 1024); w_{2^13}^j (j < 1024) then w_8^j (j < 8)
    const void *twiddles_large_lo = nullptr;
    const void *twiddles_large_hi = nullptr;
};

// Returns the cached info for the current device, initialising it (and the
// twiddle table) on first use.  nullptr + ppx error on failure.
const DeviceInfo *device_info();
// The current device's info if it has already been initialised, else nullptr
// (never touches the HIP runtime before a device has been initialised).
const DeviceInfo *device_info_if_ready();
// LDS bytes per workgroup usable by a validity check: the device's value if
// a device has been initialised in this process, else the static figure.
int64_t lds_limit();
// hipGetDevice() if this process has initialised a device through
// device_info(), else 0 without touching the HIP runtime.
int current_device_or_zero();

// ---- shape helpers ----
inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
inline int ilog2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

// ---- LDS footprint of each kernel family (bytes per workgroup) ----
int64_t fft_lds_bytes(int n, int gb, int algo, int radix);
int64_t scan_lds_bytes(int n, int gb, int P, int dtype);
int64_t tridiag_lds_bytes(int n, const ppx_config &c, int dtype);

// ---- kernel launchers (validated arguments only) ----
constexpr int kFftLog2NMax = 14;
// Workgroup-size bound of the FFT kernel holding P complex values per thread:
// at P = 32 the 64 data registers plus twiddles need more than the 128 VGPRs
// a 1024-thread workgroup leaves per lane, so those kernels cap L at 512.
constexpr int fft_max_threads(int P) { return P >= 32 ? 512 : 1024; }
// Limits of the in-wave tridiagonal kernels (registers hold P equations of
// four coefficients; PCR needs twice that again for the neighbours).
constexpr int kTriWaveMaxThreads = 256;
constexpr int tri_wave_max_p(int, int) { return 16; }
// The variant without the persistent flag, in-wave variants (registers +
// lane exchange) and the algorithm family.
constexpr int tri_base(int algo) { return algo & ~PPX_TRI_PIPE; }
constexpr bool tri_in_wave(int algo) { return tri_base(algo) >= PPX_TRI_CR_PCR; }
constexpr int tri_family(int algo) {
    return tri_base(algo) == PPX_TRI_CR || tri_base(algo) == PPX_TRI_CR_SHFL ? PPX_TRI_CR
           : tri_base(algo) == PPX_TRI_PCR || tri_base(algo) == PPX_TRI_PCR_SHFL ||
                   tri_base(algo) == PPX_TRI_PCR_REG
               ? PPX_TRI_PCR
               : tri_base(algo);  // the hybrid, WM and LF are families of one variant
}
// Families a tridiagonal tuning or job may name.
constexpr bool tri_is_family(int algo) {
    return algo == PPX_TRI_CR || algo == PPX_TRI_PCR || algo == PPX_TRI_CR_PCR || algo == PPX_TRI_WM ||
           algo == PPX_TRI_LF;
}
// Largest variant code without the persistent flag.
constexpr int kTriMaxBase = PPX_TRI_LF;
// The CR -> PCR hybrid also runs systems that span several waves (64 < n / P
// <= 1024) in one workgroup, the lanes exchanging through LDS.  Workgroup
// size bound of that kernel: 16 doubles per lane and array need more than the
// 128 VGPRs a 1024-thread workgroup leaves per lane (it spilled), so those
// shapes take at most 512 threads.
constexpr int tri_blk_max_threads(int elem_bytes, int P) { return elem_bytes * P > 64 ? 512 : 1024; }
constexpr int kTriBlkMaxLanes = 1024;
// Whether a configuration is the multi-wave hybrid.
constexpr bool tri_blk(int algo, int64_t n, int64_t P) {
    return (algo & ~PPX_TRI_PIPE) == PPX_TRI_CR_PCR && P > 0 && n / P > kWave;
}
// Largest P * sizeof(element) of the persistent in-wave variants (the second
// register set): every in-wave P.  With 16 values per lane and array the two
// register sets need 135-218 VGPRs in float32 (two or three waves per SIMD)
// and, in float64, AGPRs as well (one wave per SIMD); a persistent grid needs
// no more waves than that, and the tuners weigh the prefetch against the
// lower occupancy.
constexpr int kTriPipeMaxBytes = 128;
int launch_fft(const void *in, void *out, int log2n, int64_t batch,
               const ppx_config &c, bool inverse, hipStream_t s);
// exclusive: each output is the sum of the inputs before it (0 first).
int launch_scan(const void *in, void *out, int log2n, int64_t batch, int dtype,
                const ppx_config &c, hipStream_t s, bool exclusive = false);
int launch_tridiag(const void *a, const void *b, const void *c, const void *d,
                   void *x, int log2n, int64_t batch, int dtype,
                   const ppx_config &cfg, hipStream_t s);

// Device function pointers for occupancy queries (nullptr if no such kernel).
const void *fft_kernel(int radix, int P, int algo, int log2n);
// Kernels specialised on log2 n for radix = P = 8 / 16 (nullptr where none).
const void *fft_spec8_kernel(int log2n, bool split, bool pipe);
const void *fft_spec16_kernel(int log2n, bool split, bool pipe);
const void *fft_spec4_kernel(int log2n, bool split);  // radix = P = 4, n = 16..64; else nullptr
// The persistent FFT variants exist for radix = P = 8 or 16.
constexpr bool fft_pipe_available(int radix, int P) { return radix == P && (P == 8 || P == 16); }
const void *scan_kernel(int dtype, int P, int algo, bool exclusive = false);
// The kernel of a tridiagonal configuration (n selects the multi-wave
// hybrid for PPX_TRI_CR_PCR with n / P > 64).
const void *tridiag_kernel(int dtype, int algo, int P, int64_t n);

// Builds the forward twiddle table for NMAX = 2^kFftLog2NMax in host memory
// (float pairs from double-precision sincos).
void fft_host_twiddles(float *out2);

// ---- large-N FFT (fft_large.hip) ----
void fft_large_host_twiddles(float *lo2, float *hi2);  // 1024 and 1032 pairs
const void *fft_tile_kernel(int radix, int log2len, int tile, bool pass_a);
bool fft_tile_shape_valid(int radix, int log2len, int tile, bool pass_a);  // a pass of column length 2^log2len
int64_t fft_tile_lds_bytes(int radix, int log2len, int tile, bool pass_a);
int launch_fft_large(const void *in, void *out, int log2n, int64_t batch, const ppx_fft_plan &p, bool inverse,
                     hipStream_t s);
int fft_plan_check(int64_t n, const ppx_fft_plan &p);  // PPX_OK or a failure with reason
std::vector<std::pair<int64_t, ppx_fft_plan>> fft_recorded_plans();  // tuned plans by n
void fft_clear_plans();
void fft_default_plan(int64_t n, ppx_fft_plan &p);
std::vector<ppx_fft_plan> fft_enumerate_plans(int64_t n);
bool fft_tuned_plan(int64_t n, ppx_fft_plan &p);
void fft_record_plan(int64_t n, const ppx_fft_plan &p);

// ---- mixed launch (fused.hip) ----
struct MixPlan;
// Validates a job for the mixed launch and plans its tiles (plan may be NULL).
int check_job(const ppx_job &j, MixPlan *plan = nullptr);
// Tiles of the jobs' mixed launch, or -1 if a job cannot be planned.
int64_t mixed_tile_count(const ppx_job *jobs, int njobs);
// Completion stages of a mixed launch, for callers that retire jobs as
// their kernels finish: right after enqueuing each kernel that completes
// jobs (a family kernel, or a direct job's call) the launch calls
// stage(arg, stream), and writes that stage's index (from 0, in launch
// order) to job_stage[i] for each job i it completes.
struct MixStageHook {
    int (*stage)(void *arg, hipStream_t s);
    void *arg;
    int *job_stage;  // one entry per job
};
// launch_mixed with an optional extra event recorded after the launch and
// optional completion stages.
int launch_mixed_impl(const ppx_job *jobs, int njobs, hipStream_t stream, hipEvent_t done_event,
                      const MixStageHook *hook = nullptr);

// ---- configuration logic (config.cpp) ----
int validate_config(int op, int dtype, int64_t n, const ppx_config &c);
void complete_config(int op, int dtype, int64_t n, ppx_config &c);
int default_config(int op, int dtype, int64_t n, ppx_config &c);
int enumerate_configs(int op, int dtype, int64_t n, ppx_config *out, int cap);
int analytical_config(int op, int dtype, int64_t n, int64_t batch, ppx_config &c);
// The configuration of a tridiagonal call restricted to one family (tuned
// entry of the family, else the analytical choice within it).
int family_config(int dtype, int64_t n, int64_t batch, int family, ppx_config &c);
// tune cache (tune.cpp): entry recorded for (op, dtype, n, any algorithm)
bool cached_config(int op, int dtype, int64_t n, ppx_config &c);
void store_cached_config(int op, int dtype, int64_t n, const ppx_config &c);

}  // namespace ppx
