// Mixed batched launch: jobs of different operations, sizes and batch counts
// processed by one persistent kernel.
//
// Every job is cut into tiles of whole problems, one tile being what one
// 1024-thread workgroup processes at once with the tile shape of its
// operation: FFT radix 16 with 16 values per thread (16384 complex values
// per tile, 16384/n problems), scan with 4 values per thread for n <= 4096
// (sub-blocks of 4096 elements, up to 16384 per tile) and n/1024 above, CR or
// PCR with as many systems as the 128 KiB LDS budget holds.  The tile shape
// depends only on (op, dtype, n), so a job's result is the same bits whatever
// else shares the launch.  Workgroups are persistent -- as many as can be
// resident -- and pull tile indices from a device counter until the tile
// table is exhausted, so every workgroup exits once the table is drained.
// The counter reset and the kernel are captured once per ring slot in a
// hipGraph; a launch writes the slot's job/tile table (one host-to-device
// copy of the used part) and replays the graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "fft_device.h"
#include "ppx_internal.h"
#include "scan_device.h"
#include "tridiag_device.h"

namespace ppx {

constexpr int kFusedThreads = 1024;
constexpr int kFusedLds = 128 * 1024;
constexpr int kFusedFftElems = 16384;       // complex values per FFT tile
constexpr int kFusedScanElems = 16384;      // elements per scan tile
constexpr int kMaxJobsPerLaunch = 1 << 14;
constexpr int kMaxTilesPerLaunch = 1 << 18;
constexpr int kSlots = 4;

struct FusedJob {  // 64 bytes
    int op, dtype, log2n, flags;  // flags: FFT 1 = inverse; scan 1 = exclusive; tridiag = algo
    long long batch;
    const void *p[4];
    void *out;
};
struct FusedTile {  // 16 bytes
    int job, count;
    long long first;
};
struct FusedHeader {
    unsigned next_tile;  // work counter
    int ntiles;
};

static_assert(sizeof(FusedJob) == 64, "job layout");
static_assert(sizeof(FusedTile) == 16, "tile layout");

__global__ void k_fused_reset(FusedHeader *hdr) {
    if (threadIdx.x == 0) hdr->next_tile = 0u;
}

// A scan tile is processed in sub-blocks of kFusedThreads * P elements (P = 4
// up to n = 4096, then n / 1024), each a whole number of problems.
template <typename T, int P, bool EXCL>
__device__ __forceinline__ void scan_tile_p(const FusedJob &j, const FusedTile &t, T *wave_tot) {
    const T *in = static_cast<const T *>(j.p[0]);
    T *out = static_cast<T *>(j.out);
    const int per = (kFusedThreads * P) >> j.log2n;  // problems per sub-block (>= 1)
    for (int s = 0; s < t.count; s += per) {
        scan_block<T, P, PPX_SCAN_KS, EXCL>(in, out, j.log2n, t.first + s, min(per, t.count - s), wave_tot);
        __syncthreads();  // wave totals are reused by the next sub-block
    }
}

template <typename T, bool EXCL>
__device__ __forceinline__ void scan_tile_x(const FusedJob &j, const FusedTile &t, T *wave_tot) {
    if (j.log2n <= 12) scan_tile_p<T, 4, EXCL>(j, t, wave_tot);
    else if (j.log2n == 13) scan_tile_p<T, 8, EXCL>(j, t, wave_tot);
    else scan_tile_p<T, 16, EXCL>(j, t, wave_tot);
}

template <typename T>
__device__ __forceinline__ void scan_tile(const FusedJob &j, const FusedTile &t, T *wave_tot) {
    if (j.flags & 1) scan_tile_x<T, true>(j, t, wave_tot);
    else scan_tile_x<T, false>(j, t, wave_tot);
}

__global__ __launch_bounds__(kFusedThreads) void k_fused(const FusedJob *__restrict__ jobs,
                                                         const FusedTile *__restrict__ tiles,
                                                         FusedHeader *hdr,
                                                         const float2 *__restrict__ tw) {
    extern __shared__ float4 lds[];
    __shared__ int s_tile;
    __shared__ double wave_tot_d[kFusedThreads / kWave];  // float and int totals alias its start
    float *wave_tot_f = reinterpret_cast<float *>(wave_tot_d);
    int *wave_tot_i = reinterpret_cast<int *>(wave_tot_d);
    const int ntiles = hdr->ntiles;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(&hdr->next_tile, 1u);
        __syncthreads();
        const int ti = s_tile;
        __syncthreads();
        if (ti >= ntiles) break;  // uniform: every wave of the workgroup leaves
        const FusedTile t = tiles[ti];
        const FusedJob j = jobs[t.job];
        if (j.op == PPX_OP_FFT) {
            fft_block<16, 16, false>(static_cast<const float2 *>(j.p[0]), static_cast<float2 *>(j.out), tw,
                                     j.log2n, t.first, t.count, (j.flags & 1) ? -1.0f : 1.0f, lds);
        } else if (j.op == PPX_OP_SCAN) {
            if (j.dtype == PPX_I32) scan_tile<int>(j, t, wave_tot_i);
            else if (j.dtype == PPX_F32) scan_tile<float>(j, t, wave_tot_f);
            else scan_tile<double>(j, t, wave_tot_d);
        } else if (j.dtype == PPX_F32) {
            const float *const *p = reinterpret_cast<const float *const *>(j.p);
            if (j.flags == PPX_TRI_PCR)
                tridiag_block<float, PPX_TRI_PCR>(p[0], p[1], p[2], p[3], static_cast<float *>(j.out),
                                                  j.log2n, t.first, t.count, reinterpret_cast<float *>(lds));
            else
                tridiag_block<float, PPX_TRI_CR>(p[0], p[1], p[2], p[3], static_cast<float *>(j.out),
                                                 j.log2n, t.first, t.count, reinterpret_cast<float *>(lds));
        } else {
            const double *const *p = reinterpret_cast<const double *const *>(j.p);
            if (j.flags == PPX_TRI_PCR)
                tridiag_block<double, PPX_TRI_PCR>(p[0], p[1], p[2], p[3], static_cast<double *>(j.out),
                                                   j.log2n, t.first, t.count, reinterpret_cast<double *>(lds));
            else
                tridiag_block<double, PPX_TRI_CR>(p[0], p[1], p[2], p[3], static_cast<double *>(j.out),
                                                  j.log2n, t.first, t.count, reinterpret_cast<double *>(lds));
        }
        __syncthreads();  // LDS and the tile index are reused by the next tile
    }
}

// ------------------------------------------------------------------- host

// Problems per tile of a job: a pure function of (op, dtype, n, algo).
int64_t fused_tile_problems(int op, int dtype, int64_t n, int algo) {
    if (op == PPX_OP_FFT) return std::max<int64_t>(1, kFusedFftElems / n);
    if (op == PPX_OP_SCAN) return std::max<int64_t>(1, kFusedScanElems / n);
    const int64_t per_sys = tri_lds_arrays(algo) * (dtype == PPX_F64 ? 8 : 4) * n;
    const int64_t by_lds = kFusedLds / per_sys;
    const int64_t by_threads = 2 * kFusedThreads / n > 0 ? 2 * kFusedThreads / n : 1;
    return std::min(by_lds, std::max<int64_t>(1, by_threads));
}

namespace {
struct Slot {
    FusedJob *d_jobs = nullptr;
    FusedTile *d_tiles = nullptr;
    FusedHeader *d_hdr = nullptr;
    char *h_stage = nullptr;  // pinned: header | jobs | tiles
    hipEvent_t done = nullptr;
    hipGraphExec_t exec = nullptr;
    bool used = false;
};
struct MixedCtx {
    int device = -1;
    int grid = 0;
    Slot slots[kSlots];
    int next = 0;
};
std::mutex g_mixed_mu;
std::vector<MixedCtx *> g_mixed;  // per device ordinal, never freed

constexpr size_t kStageBytes = 256 + sizeof(FusedJob) * kMaxJobsPerLaunch + sizeof(FusedTile) * kMaxTilesPerLaunch;

int init_ctx(MixedCtx *m, const DeviceInfo *di) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fused),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kFusedLds);
    (void)e;  // not every runtime needs it; the occupancy query below decides
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused, kFusedThreads, kFusedLds) != hipSuccess ||
        per_cu < 1)
        return fail(PPX_EHIP, "fused kernel cannot be resident");
    m->grid = per_cu * di->cus;
    hipStream_t cap;
    if (hipStreamCreate(&cap) != hipSuccess) return fail(PPX_EHIP, "stream creation failed");
    for (auto &s : m->slots) {
        if (hipMalloc(&s.d_hdr, 256) != hipSuccess ||
            hipMalloc(&s.d_jobs, sizeof(FusedJob) * kMaxJobsPerLaunch) != hipSuccess ||
            hipMalloc(&s.d_tiles, sizeof(FusedTile) * kMaxTilesPerLaunch) != hipSuccess ||
            hipHostMalloc(&s.h_stage, kStageBytes, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
            return fail(PPX_ENOMEM, "could not allocate the mixed-launch tables");
        // capture: counter reset, then the persistent kernel, reading this
        // slot's tables at fixed addresses
        hipGraph_t g;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(PPX_EHIP, "graph capture failed");
        hipLaunchKernelGGL(k_fused_reset, dim3(1), dim3(64), 0, cap, s.d_hdr);
        hipLaunchKernelGGL(k_fused, dim3(m->grid), dim3(kFusedThreads), kFusedLds, cap, s.d_jobs,
                           s.d_tiles, s.d_hdr, static_cast<const float2 *>(di->twiddles));
        if (hipStreamEndCapture(cap, &g) != hipSuccess) return fail(PPX_EHIP, "graph capture failed");
        const hipError_t ie = hipGraphInstantiate(&s.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return fail(PPX_EHIP, "graph instantiation failed");
    }
    (void)hipStreamDestroy(cap);
    return PPX_OK;
}

MixedCtx *mixed_ctx() {
    const DeviceInfo *di = device_info();
    if (!di) return nullptr;
    std::lock_guard<std::mutex> lk(g_mixed_mu);
    if ((int)g_mixed.size() <= di->device) g_mixed.resize(di->device + 1, nullptr);
    if (!g_mixed[di->device]) {
        auto *m = new MixedCtx();
        m->device = di->device;
        if (init_ctx(m, di) != PPX_OK) return nullptr;  // leaks the partial context on purpose
        g_mixed[di->device] = m;
    }
    return g_mixed[di->device];
}
}  // namespace

// Validates one job against the single-call rules and the fused limits.
int check_job(const ppx_job &j) {
    if (!j.in || !j.out) return fail(PPX_EINVAL, "job: null pointer");
    if (!is_pow2(j.n) || j.n < PPX_MIN_N || j.n > PPX_MAX_N) return fail(PPX_EINVAL, "job: bad n");
    if (j.batch < 1) return fail(PPX_EINVAL, "job: batch must be >= 1");
    auto al = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    if (!al(j.in) || !al(j.out)) return fail(PPX_EINVAL, "job: pointers must be 16-byte aligned");
    switch (j.op) {
        case PPX_OP_FFT:
            if (j.dtype != PPX_C64 || (j.direction != -1 && j.direction != 1))
                return fail(PPX_EINVAL, "job: FFT needs dtype PPX_C64 and direction -1/+1");
            break;
        case PPX_OP_SCAN:
            if (j.dtype != PPX_I32 && j.dtype != PPX_F32 && j.dtype != PPX_F64)
                return fail(PPX_EINVAL, "job: scan dtype");
            if (j.algo != PPX_JOB_SCAN_INCLUSIVE && j.algo != PPX_JOB_SCAN_EXCLUSIVE)
                return fail(PPX_EINVAL, "job: scan algo must be PPX_JOB_SCAN_INCLUSIVE or _EXCLUSIVE");
            break;
        case PPX_OP_TRIDIAG: {
            if (j.dtype != PPX_F32 && j.dtype != PPX_F64) return fail(PPX_EINVAL, "job: tridiagonal dtype");
            if (j.algo != PPX_TRI_CR && j.algo != PPX_TRI_PCR) return fail(PPX_EINVAL, "job: tridiagonal algo");
            if (!j.b || !j.c || !j.d || !al(j.b) || !al(j.c) || !al(j.d))
                return fail(PPX_EINVAL, "job: tridiagonal coefficient pointers");
            const int64_t per_sys = tri_lds_arrays(j.algo) * (j.dtype == PPX_F64 ? 8 : 4) * j.n;
            if (per_sys > kFusedLds) return fail(PPX_EINVAL, "job: tridiagonal system too large for a fused tile");
            break;
        }
        default:
            return fail(PPX_EINVAL, "job: unknown op");
    }
    return PPX_OK;
}

int64_t mixed_tile_count(const ppx_job *jobs, int njobs) {
    int64_t tiles = 0;
    for (int i = 0; i < njobs; ++i) {
        const int64_t per = fused_tile_problems(jobs[i].op, jobs[i].dtype, jobs[i].n, jobs[i].algo);
        tiles += (jobs[i].batch + per - 1) / per;
    }
    return tiles;
}

int launch_mixed_impl(const ppx_job *jobs, int njobs, hipStream_t stream, hipEvent_t done_event) {
    if (!jobs || njobs < 1) return fail(PPX_EINVAL, "no jobs");
    if (njobs > kMaxJobsPerLaunch) return fail(PPX_EINVAL, "too many jobs for one mixed launch");
    for (int i = 0; i < njobs; ++i)
        if (int rc = check_job(jobs[i])) return rc;
    const int64_t ntiles = mixed_tile_count(jobs, njobs);
    if (ntiles > kMaxTilesPerLaunch) return fail(PPX_EINVAL, "too many tiles for one mixed launch");
    MixedCtx *m = mixed_ctx();
    if (!m) return PPX_EHIP;
    std::unique_lock<std::mutex> lk(g_mixed_mu);
    Slot &s = m->slots[m->next];
    m->next = (m->next + 1) % kSlots;
    if (s.used && hipEventSynchronize(s.done) != hipSuccess) return fail(PPX_EHIP, "slot wait failed");
    // host tables in the slot's pinned staging buffer
    auto *hdr = reinterpret_cast<FusedHeader *>(s.h_stage);
    auto *hj = reinterpret_cast<FusedJob *>(s.h_stage + 256);
    auto *ht = reinterpret_cast<FusedTile *>(s.h_stage + 256 + sizeof(FusedJob) * kMaxJobsPerLaunch);
    int64_t k = 0;
    for (int i = 0; i < njobs; ++i) {
        const ppx_job &j = jobs[i];
        FusedJob &f = hj[i];
        f.op = j.op;
        f.dtype = j.dtype;
        f.log2n = ilog2(j.n);
        f.flags = j.op == PPX_OP_FFT ? (j.direction == 1 ? 1 : 0) : j.algo;  // scan: exclusive; tridiag: algo
        f.batch = j.batch;
        f.p[0] = j.in;
        f.p[1] = j.b;
        f.p[2] = j.c;
        f.p[3] = j.d;
        f.out = j.out;
        const int64_t per = fused_tile_problems(j.op, j.dtype, j.n, j.algo);
        for (int64_t p = 0; p < j.batch; p += per) {
            ht[k].job = i;
            ht[k].count = (int)std::min<int64_t>(per, j.batch - p);
            ht[k].first = p;
            ++k;
        }
    }
    hdr->next_tile = 0;
    hdr->ntiles = (int)ntiles;
    hipError_t e = hipMemcpyAsync(s.d_hdr, hdr, sizeof(FusedHeader), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.d_jobs, hj, sizeof(FusedJob) * njobs, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.d_tiles, ht, sizeof(FusedTile) * ntiles, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipGraphLaunch(s.exec, stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, stream);
    if (e == hipSuccess && done_event) e = hipEventRecord(done_event, stream);
    s.used = true;
    return fail_hip(e, "mixed launch");
}

}  // namespace ppx

extern "C" int launch_mixed(const ppx_job *jobs, int njobs, void *stream) {
    ppx::fail(PPX_OK, "");
    return ppx::launch_mixed_impl(jobs, njobs, static_cast<hipStream_t>(stream), nullptr);
}

extern "C" int ppx_mixed_tile_problems(int op, int dtype, int64_t n, int algo) {
    return (int)ppx::fused_tile_problems(op, dtype, n, algo);
}
