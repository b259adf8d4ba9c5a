// Mixed batched launch, host side: planning each job's tiles from its tuned
// configuration, the launch tables, and the launches of the family kernels
// (see mixed.h).
//
// A launch with at most kMixArgJobs jobs in every family passes each
// family's job records in the kernel arguments: one kernel launch per
// family, a workgroup per tile, nothing else.  Any other launch copies one
// table (header and job records) from pinned memory to the device and
// enqueues [expand the tile lists] -> [family kernel] -> ..., each family
// kernel persistent (at most as many workgroups as are resident, and no more
// than its tiles), draining its family's tiles, so every workgroup exits
// once they are done.  Either way the families go in ascending order of
// their jobs' elements, and the jobs that run as their own calls last.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mixed.h"
#include "tridiag_device.h"

namespace ppx {

constexpr int kSlots = 4;

int64_t mix_lds_bytes(int fam) {
    switch (fam) {
        case kFamFft256: return 256 * 16 * 8;    // complex exchange, P = 16
        case kFamFft1024: return 1024 * 16 * 8;  // complex exchange, P = 16
        case kFamFft1024P8: return 1024 * 8 * 8;  // complex exchange, P = 8
        case kFamTriW32: return 0;  // no PCR exchange, no staged stores (P <= 8)
        case kFamTriW32H: return 4 * 64 * 16 * 4;  // per wave: PCR exchange (3 * 64 * 4) or P = 16 staging (64 * 16) floats
        case kFamTriW64: return 4 * 3 * 64 * 4 * 8;  // per wave: PCR exchange (3 * 64 * 4) or P = 8 staging (64 * 8) doubles
        case kFamTriW64H: return 4 * 64 * 16 * 8;    // per wave: P = 16 staging (64 * 16 doubles) or PCR exchange (3 * 64 * 4)
        case kFamTriLds: return kMixTriLdsBudget;
        case kFamTriBlk32:
        case kFamTriBlk32H: return 6 * 1024 * 4;  // two sets of a, c, d lane slots
        case kFamTriBlk64: return 6 * 1024 * 8;
        case kFamTriBlk64H: return 6 * 512 * 8;
        default: return 0;  // scan: static wave-total slots only
    }
}

// The family's kernel (persistent, or taking its records in the arguments),
// from whichever translation unit instantiates it.
static const void *mix_kernel(int fam, bool args) {
    if (const void *k = mix_fft_kernel(fam, args)) return k;
    if (const void *k = mix_scan_kernel(fam, args)) return k;
    return mix_tri_kernel(fam, args);
}

// Writes each job's run of its family's tile list: entry first_tile + k of
// the job's family is the job's index, k < the job's tile count.
__global__ __launch_bounds__(kMixExpandThreads) void k_mix_expand(char *tables) {
    const MixHeader *h = reinterpret_cast<const MixHeader *>(tables);
    const MixJob *jobs = reinterpret_cast<const MixJob *>(tables + kMixHeaderBytes);
    unsigned *tiles = reinterpret_cast<unsigned *>(tables + h->tiles_off);
    const unsigned njobs = h->njobs;
    for (unsigned jb = blockIdx.x; jb < njobs; jb += gridDim.x) {
        const MixJob &j = jobs[jb];
        const unsigned nt = (unsigned)((j.batch + j.per_tile - 1) / j.per_tile);
        unsigned *dst = tiles + h->tile_base[j.family] + j.first_tile;
        for (unsigned k = threadIdx.x; k < nt; k += blockDim.x) dst[k] = jb;
    }
}

const void *mix_expand_kernel() { return reinterpret_cast<const void *>(&k_mix_expand); }

// ------------------------------------------------------------- planning

// The configuration the single call with cfg == NULL uses for this job: the
// tuned (or analytical) one for (op, dtype, n); for a tridiagonal job, the
// one of its family (the job's algo).
int job_config(const ppx_job &j, ppx_config &c) {
    if (j.op == PPX_OP_TRIDIAG) return family_config(j.dtype, j.n, j.batch, j.algo, c);
    const int dtype = j.op == PPX_OP_FFT ? PPX_C64 : j.dtype;
    if (ppx_resolve_config(j.op, dtype, j.n, j.batch, &c) != PPX_OK) return PPX_ECONFIG;
    return PPX_OK;
}

// Radix = P = 8 or 16, or 4 up to n = 1024: the shapes the FFT families hold.
static bool fft_mix_shape(int radix, int P, int64_t n) {
    return radix == P && (P == 8 || P == 16 || (P == 4 && n <= 1024));
}

int mix_plan(const ppx_job &j, MixPlan &m) {
    ppx_config c;
    if (int rc = job_config(j, c)) return rc;
    const int log2n = ilog2(j.n);
    m.flags = 0;
    const int pipe = j.op == PPX_OP_FFT ? PPX_FFT_LDS_PIPE : j.op == PPX_OP_SCAN ? PPX_SCAN_KS_PIPE : PPX_TRI_PIPE;
    if ((c.algo & pipe) && j.n * j.batch >= PPX_MIXED_DIRECT_ELEMS) {
        m.direct = true;
        m.family = m.shape = -1;
        m.per_tile = c.problems_per_block;
        m.tpp = 0;
        m.block = c.threads_per_block;
        m.ntiles = 0;
        m.cfg = c;
        return PPX_OK;
    }
    m.direct = false;
    if (j.op == PPX_OP_FFT) {
        c.algo &= ~PPX_FFT_LDS_PIPE;  // the launch is persistent itself
        if (!fft_mix_shape(c.radix, c.elems_per_thread, j.n)) {
            // a shape the families do not hold: the nearest radix = P one, at
            // one problem per 64-thread group at least
            const int P = (c.elems_per_thread <= 8 && j.n / 8 <= kMaxThreadsPerBlock) ? 8 : 16;
            const int64_t T = j.n / P;
            c.radix = P;
            c.elems_per_thread = P;
            c.problems_per_block = (int)std::max<int64_t>(1, kWave / T);
            c.threads_per_block = (int)(T * c.problems_per_block);
            c.lds_elems = 0;
            complete_config(PPX_OP_FFT, PPX_C64, j.n, c);
            if (validate_config(PPX_OP_FFT, PPX_C64, j.n, c)) return fail(PPX_ECONFIG, "job: no FFT tile shape");
        }
        const int P = c.elems_per_thread;
        const int64_t T = j.n / P;
        m.family = T <= 256 ? kFamFft256 : P == 8 ? kFamFft1024P8 : kFamFft1024;
        const bool split = (c.algo & PPX_FFT_LDS_SPLIT) != 0;
        m.shape = mix_fft_shape(log2n, P, split);
        m.tpp = (int)T;
        m.flags = j.direction == 1 ? 1 : 0;
    } else if (j.op == PPX_OP_SCAN) {
        c.algo &= PPX_SCAN_LF;  // KS or LF; the persistent flag cleared
        const int P = c.elems_per_thread;
        const int64_t T = j.n / P;
        m.family = T <= 256 ? kFamScan256 : kFamScan1024;
        m.shape = mix_scan_shape(j.dtype, ilog2(P), c.algo == PPX_SCAN_LF);
        m.tpp = (int)T;
        m.flags = j.algo == PPX_JOB_SCAN_EXCLUSIVE ? 1 : 0;
    } else {
        c.algo = tri_base(c.algo);
        const bool f64 = j.dtype == PPX_F64;
        if (tri_blk(c.algo, j.n, c.elems_per_thread)) {  // the hybrid across waves
            const int P = c.elems_per_thread;
            m.family = !f64 ? (P == 16 ? kFamTriBlk32H : kFamTriBlk32) : P == 16 ? kFamTriBlk64H : kFamTriBlk64;
            m.shape = ilog2(P) - 1;
            m.tpp = (int)(j.n / P);
        } else if (tri_in_wave(c.algo)) {
            const int P = c.elems_per_thread;
            m.family = mix_triw_family(f64, c.algo, P);
            m.shape = mix_triw_shape(c.algo, ilog2(P));
            m.tpp = (int)(j.n / P);
        } else {
            const int64_t per_sys = tri_lds_arrays(c.algo) * (f64 ? 8 : 4) * j.n;
            if (per_sys > kMixTriLdsBudget)
                return fail(PPX_EINVAL, "job: tridiagonal system too large for a mixed-launch tile (128 KiB of LDS)");
            const int64_t scaled = (int64_t)c.problems_per_block * 1024 / c.threads_per_block;
            m.family = kFamTriLds;
            m.shape = mix_tril_shape(f64, c.algo == PPX_TRI_PCR);
            m.per_tile = (int)std::max<int64_t>(1, std::min<int64_t>(scaled, kMixTriLdsBudget / per_sys));
            m.tpp = 0;  // its tiles are sized by LDS, in 1024-thread workgroups
        }
    }
    m.cfg = c;
    // the tuned workgroup size, within what the family's kernel allows and
    // at least a wave and a problem's threads
    m.block = m.tpp ? std::min(mix_block(m.family), std::max({c.threads_per_block, m.tpp, kWave})) : mix_block(m.family);
    if (m.tpp) m.per_tile = m.block / m.tpp;
    m.ntiles = (j.batch + m.per_tile - 1) / m.per_tile;
    return PPX_OK;
}

// Validates one job against the single-call rules and the mixed-launch
// limits, and plans its tiles.
int check_job(const ppx_job &j, MixPlan *plan) {
    if (!j.in || !j.out) return fail(PPX_EINVAL, "job: null pointer");
    if (!is_pow2(j.n) || j.n < PPX_MIN_N || j.n > PPX_MAX_N) return fail(PPX_EINVAL, "job: bad n");
    if (j.batch < 1) return fail(PPX_EINVAL, "job: batch must be >= 1");
    if (j.batch > (int64_t(1) << 40) / j.n) return fail(PPX_EINVAL, "job: batch * n is too large");
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
        case PPX_OP_TRIDIAG:
            if (j.dtype != PPX_F32 && j.dtype != PPX_F64) return fail(PPX_EINVAL, "job: tridiagonal dtype");
            if (!tri_is_family(j.algo))
                return fail(PPX_EINVAL, "job: tridiagonal algo must be a family: PPX_TRI_CR, _PCR, _CR_PCR, _WM or _LF");
            if (!j.b || !j.c || !j.d || !al(j.b) || !al(j.c) || !al(j.d))
                return fail(PPX_EINVAL, "job: tridiagonal coefficient pointers");
            break;
        default:
            return fail(PPX_EINVAL, "job: unknown op");
    }
    MixPlan m;
    if (int rc = mix_plan(j, m)) return rc;
    if (m.ntiles > kMixMaxTiles) return fail(PPX_EINVAL, "job: more tiles than one mixed launch holds");
    if (plan) *plan = m;
    return PPX_OK;
}

int64_t mixed_tile_count(const ppx_job *jobs, int njobs) {
    int64_t tiles = 0;
    for (int i = 0; i < njobs; ++i) {
        MixPlan m;
        if (mix_plan(jobs[i], m) != PPX_OK) return -1;
        tiles += m.ntiles;
    }
    return tiles;
}

// Plans every job and writes the header and job records into `buf` (at
// least mix_table_bytes(njobs, 0) bytes).  Returns the family mask, or a
// negative error.  ntiles_out receives the total tile count.
int mix_build_tables(const ppx_job *jobs, int njobs, char *buf, int64_t *ntiles_out, int *direct, int *ndirect,
                     int *rec_job) {
    if (!jobs || njobs < 1) return fail(PPX_EINVAL, "no jobs");
    if (njobs > kMixMaxJobs) return fail(PPX_EINVAL, "too many jobs for one mixed launch");
    auto *h = reinterpret_cast<MixHeader *>(buf);
    auto *rec = reinterpret_cast<MixJob *>(buf + kMixHeaderBytes);
    std::memset(h, 0, kMixHeaderBytes);
    int nrec = 0;
    *ndirect = 0;
    // pass 1: plan every job; a record's per_tile holds its problem's
    // threads until the family's workgroup size is known (the largest of its
    // jobs' tuned sizes)
    for (int i = 0; i < njobs; ++i) {
        MixPlan m;
        if (int rc = check_job(jobs[i], &m)) return rc;
        if (m.direct) {
            direct[(*ndirect)++] = i;
            continue;
        }
        const ppx_job &j = jobs[i];
        MixJob &r = rec[nrec];
        r.shape = m.shape;
        r.flags = m.flags;
        r.log2n = ilog2(j.n);
        r.per_tile = m.tpp ? m.tpp : m.per_tile;
        r.batch = j.batch;
        r.first_tile = 0;
        r.family = m.family;
        r.p[0] = j.in;
        r.p[1] = j.b;
        r.p[2] = j.c;
        r.p[3] = j.d;
        r.out = j.out;
        h->block[m.family] = std::max<unsigned>(h->block[m.family], (unsigned)m.block);
        if (rec_job) rec_job[nrec] = i;
        ++nrec;
    }
    // pass 2: problems per tile at the family's workgroup size, tile ranges
    int64_t fam_tiles[kMixFamilies] = {};
    for (int k = 0; k < nrec; ++k) {
        MixJob &r = rec[k];
        if (r.family != kFamTriLds) r.per_tile = (int)h->block[r.family] / r.per_tile;
        r.first_tile = (unsigned)fam_tiles[r.family];
        fam_tiles[r.family] += (r.batch + r.per_tile - 1) / r.per_tile;
        if (fam_tiles[r.family] > kMixMaxTiles) return fail(PPX_EINVAL, "too many tiles for one mixed launch");
    }
    int64_t total = 0;
    int mask = 0;
    for (int f = 0; f < kMixFamilies; ++f) {
        h->tile_base[f] = (unsigned)total;
        h->ntiles[f] = (unsigned)fam_tiles[f];
        total += fam_tiles[f];
        if (fam_tiles[f]) mask |= 1 << f;
    }
    if (total > kMixMaxTiles) return fail(PPX_EINVAL, "too many tiles for one mixed launch");
    h->njobs = (unsigned)nrec;
    h->tiles_off = (unsigned)((kMixHeaderBytes + (int64_t)nrec * sizeof(MixJob) + 15) & ~int64_t(15));
    *ntiles_out = total;
    return mask;
}

// ------------------------------------------------------- device context
namespace {
struct Slot {
    char *d_tables = nullptr;
    char *h_stage = nullptr;  // pinned: header | jobs
    hipEvent_t done = nullptr;
    bool used = false;
};
struct MixedCtx {
    int device = -1;
    Slot slots[kSlots];
    int next = 0;
    std::vector<char> plan;  // host tables of the launch being planned
};
std::mutex g_mixed_mu;
std::vector<MixedCtx *> g_mixed;  // per device ordinal, never freed

constexpr size_t kTableBytes = (size_t)mix_table_bytes(kMixMaxJobs, kMixMaxTiles) + 16;
constexpr size_t kStageBytes = (size_t)mix_table_bytes(kMixMaxJobs, 0);

int init_ctx(MixedCtx *m) {
    if (int rc = mix_prepare_kernels()) return rc;
    for (auto &s : m->slots) {
        if (hipMalloc(&s.d_tables, kTableBytes) != hipSuccess ||
            hipHostMalloc(&s.h_stage, kStageBytes, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
            return fail(PPX_ENOMEM, "could not allocate the mixed-launch tables");
    }
    m->plan.resize(kStageBytes);
    return PPX_OK;
}

MixedCtx *mixed_ctx() {
    const DeviceInfo *di = device_info();
    if (!di) return nullptr;
    if ((int)g_mixed.size() <= di->device) g_mixed.resize(di->device + 1, nullptr);
    if (!g_mixed[di->device]) {
        auto *m = new MixedCtx();
        m->device = di->device;
        if (init_ctx(m) != PPX_OK) return nullptr;  // leaks the partial context on purpose
        g_mixed[di->device] = m;
    }
    return g_mixed[di->device];
}
}  // namespace

// Resident workgroups of each family's persistent kernel on the current
// device at each workgroup size 64 << k up to the family's (from the
// occupancy query at that size and its LDS), set up once per process.
constexpr int kMixBlockSizes = 5;  // 64 .. 1024
static int g_resident[kMixFamilies][kMixBlockSizes];

// LDS bytes of family fam's kernel at workgroup size block: the tiles'
// buffers scale with it, except the LDS-exchange tridiagonal family's.
static size_t mix_lds_at(int fam, int block) {
    return fam == kFamTriLds ? (size_t)mix_lds_bytes(fam) : (size_t)(mix_lds_bytes(fam) * block / mix_block(fam));
}
static bool g_prepared = false;
static std::mutex g_prep_mu;

int mix_prepare_kernels() {
    std::lock_guard<std::mutex> lk(g_prep_mu);
    if (g_prepared) return PPX_OK;
    const DeviceInfo *di = device_info();
    if (!di) return PPX_EDEVICE;
    for (int f = 0; f < kMixFamilies; ++f) {
        for (int args = 0; args < 2; ++args) {
            const void *k = mix_kernel(f, args != 0);
            if (!k) return fail(PPX_EHIP, "mixed launch: no kernel for family " + std::to_string(f));
            (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mix_lds_bytes(f));
            for (int b = 0; b < kMixBlockSizes && (kWave << b) <= mix_block(f); ++b) {
                const int block = kWave << b;
                int per_cu = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, mix_lds_at(f, block)) !=
                        hipSuccess ||
                    per_cu < 1)
                    return fail(PPX_EHIP,
                                "mixed launch: the kernel of family " + std::to_string(f) + " cannot be resident");
                if (!args) g_resident[f][b] = per_cu * di->cus;
            }
        }
    }
    g_prepared = true;
    return PPX_OK;
}

// Enqueues the expansion and the kernels of the families in `mask` on
// stream s, reading the tables at d_tables; each family's grid is its
// resident count capped at its tile count ntiles[f].
int mix_enqueue(char *d_tables, int mask, const int64_t *ntiles, const unsigned *blocks, const int *order, int norder,
                const float2 *tw, hipStream_t s, mix_after_family_t after, void *arg) {
    hipLaunchKernelGGL(k_mix_expand, dim3(kMixExpandBlocks), dim3(kMixExpandThreads), 0, s, d_tables);
    hipError_t e = hipGetLastError();
    MixArgs a;
    a.tables = d_tables;
    a.ntiles = a.njobs = 0;
    for (int k = 0; k < norder && e == hipSuccess; ++k) {
        const int f = order[k];
        if (!(mask & (1 << f))) continue;
        const int block = (int)blocks[f];
        const int64_t grid = std::min<int64_t>(g_resident[f][ilog2(block / kWave)], std::max<int64_t>(1, ntiles[f]));
        hipLaunchKernelGGL(reinterpret_cast<mix_kernel_t>(const_cast<void *>(mix_kernel(f, false))), dim3((unsigned)grid),
                           dim3(block), mix_lds_at(f, block), s, a, tw);
        e = hipGetLastError();
        if (e == hipSuccess && after)
            if (int rc = after(arg, f, s)) return rc;
    }
    return fail_hip(e, "mixed launch");
}

int mix_family_order(const char *table, int mask, int *order) {
    const MixHeader *h = reinterpret_cast<const MixHeader *>(table);
    const MixJob *rec = reinterpret_cast<const MixJob *>(table + kMixHeaderBytes);
    double work[kMixFamilies] = {};
    for (unsigned i = 0; i < h->njobs; ++i) work[rec[i].family] += std::ldexp(double(rec[i].batch), rec[i].log2n);
    int n = 0;
    for (int f = 0; f < kMixFamilies; ++f)
        if (mask & (1 << f)) order[n++] = f;
    std::stable_sort(order, order + n, [&](int x, int y) { return work[x] < work[y]; });
    return n;
}

bool mix_args_fit(const char *table, int mask) {
    const MixHeader *h = reinterpret_cast<const MixHeader *>(table);
    const MixJob *rec = reinterpret_cast<const MixJob *>(table + kMixHeaderBytes);
    int per_family[kMixFamilies] = {};
    for (unsigned i = 0; i < h->njobs; ++i) ++per_family[rec[i].family];
    for (int f = 0; f < kMixFamilies; ++f)
        if ((mask & (1 << f)) && per_family[f] > kMixArgJobs) return false;
    return true;
}

// Workgroups an argument launch aims for at least before it shrinks tiles:
// four per CU (one per SIMD).
constexpr int kMixFillPerCu = 4;

int mix_enqueue_args(const char *table, int mask, const int *order, int norder, const float2 *tw, hipStream_t s,
                     mix_after_family_t after, void *arg) {
    const MixHeader *h = reinterpret_cast<const MixHeader *>(table);
    const MixJob *rec = reinterpret_cast<const MixJob *>(table + kMixHeaderBytes);
    // A launch with fewer full tiles than it takes to fill the GPU runs its
    // families in smaller workgroups (a problem's threads and arithmetic
    // unchanged, fewer problems per tile), which spreads small batches over
    // more CUs; the LDS-exchange tridiagonal family keeps its shape.
    int64_t total = 0;
    for (int f = 0; f < kMixFamilies; ++f)
        if (mask & (1 << f)) total += h->ntiles[f];
    const int64_t fill = (int64_t)kMixFillPerCu * device_info()->cus;
    int shrink = 1;
    while (shrink < 1024 && total * shrink * 2 <= fill) shrink *= 2;
    hipError_t e = hipSuccess;
    for (int o = 0; o < norder && e == hipSuccess; ++o) {
        const int f = order[o];
        if (!(mask & (1 << f))) continue;
        const int full = (int)h->block[f];
        int block = full;
        if (shrink > 1 && f != kFamTriLds) {
            int need = kWave;  // threads of the widest problem among the family's jobs
            for (unsigned i = 0; i < h->njobs; ++i)
                if (rec[i].family == f) need = std::max(need, full / rec[i].per_tile);
            block = std::max(full / shrink, need);
        }
        MixArgs a;
        a.tables = nullptr;
        a.ntiles = 0;
        a.njobs = 0;
        for (unsigned i = 0; i < h->njobs; ++i) {
            if (rec[i].family != f) continue;
            MixJob r = rec[i];  // first_tile ascending, as the kernel scans them
            r.per_tile = (int)((int64_t)r.per_tile * block / full);
            r.first_tile = a.ntiles;
            a.ntiles += (unsigned)((r.batch + r.per_tile - 1) / r.per_tile);
            a.jobs[a.njobs++] = r;
        }
        const size_t lds = mix_lds_at(f, block);
        hipLaunchKernelGGL(reinterpret_cast<mix_kernel_t>(const_cast<void *>(mix_kernel(f, true))), dim3(a.ntiles),
                           dim3(block), lds, s, a, tw);
        e = hipGetLastError();
        if (e == hipSuccess && after)
            if (int rc = after(arg, f, s)) return rc;
    }
    return fail_hip(e, "mixed launch");
}

namespace {
// Stage bookkeeping of one launch: which records each family completes.
struct StageCtx {
    const MixStageHook *hook;
    const MixJob *rec;
    const int *rec_job;
    unsigned nrec;
    int next;
};
int after_family(void *arg, int fam, hipStream_t s) {
    auto *c = static_cast<StageCtx *>(arg);
    for (unsigned r = 0; r < c->nrec; ++r)
        if (c->rec[r].family == fam) c->hook->job_stage[c->rec_job[r]] = c->next;
    ++c->next;
    return c->hook->stage(c->hook->arg, s);
}
}  // namespace

int launch_mixed_impl(const ppx_job *jobs, int njobs, hipStream_t stream, hipEvent_t done_event,
                      const MixStageHook *hook) {
    if (!jobs || njobs < 1) return fail(PPX_EINVAL, "no jobs");
    if (njobs > kMixMaxJobs) return fail(PPX_EINVAL, "too many jobs for one mixed launch");
    std::unique_lock<std::mutex> lk(g_mixed_mu);
    MixedCtx *m = mixed_ctx();
    if (!m) return PPX_EHIP;
    int64_t ntiles = 0;
    std::vector<int> direct(njobs), rec_job(njobs);
    int ndirect = 0;
    char *table = m->plan.data();
    const int mask = mix_build_tables(jobs, njobs, table, &ntiles, direct.data(), &ndirect, rec_job.data());
    if (mask < 0) return mask;
    direct.resize(ndirect);
    const MixHeader *h = reinterpret_cast<const MixHeader *>(table);
    StageCtx sc{hook, reinterpret_cast<const MixJob *>(table + kMixHeaderBytes), rec_job.data(), h->njobs, 0};
    const mix_after_family_t after = hook ? after_family : nullptr;
    int order[kMixFamilies];
    const int norder = mix_family_order(table, mask, order);
    const float2 *tw = static_cast<const float2 *>(device_info()->twiddles);
    hipError_t e = hipSuccess;
    if (mask && mix_args_fit(table, mask)) {  // the records go in the kernel arguments
        if (int rc = mix_enqueue_args(table, mask, order, norder, tw, stream, after, &sc)) return rc;
    } else if (mask) {  // the tiled jobs: one table copy, the expansion and the family kernels
        Slot &s = m->slots[m->next];
        if (s.used && hipEventSynchronize(s.done) != hipSuccess) return fail(PPX_EHIP, "slot wait failed");
        m->next = (m->next + 1) % kSlots;
        const size_t bytes = kMixHeaderBytes + (size_t)h->njobs * sizeof(MixJob);
        std::memcpy(s.h_stage, table, bytes);
        int64_t fam_tiles[kMixFamilies];
        for (int f = 0; f < kMixFamilies; ++f) fam_tiles[f] = h->ntiles[f];
        e = hipMemcpyAsync(s.d_tables, s.h_stage, bytes, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return fail_hip(e, "mixed launch");
        if (int rc = mix_enqueue(s.d_tables, mask, fam_tiles, h->block, order, norder, tw, stream, after, &sc))
            return rc;
        e = hipEventRecord(s.done, stream);
        s.used = true;
        if (e != hipSuccess) return fail_hip(e, "mixed launch");
    }
    for (int i : direct) {  // jobs that fill the GPU alone: their tuned single calls, after the tiles
        MixPlan p;
        (void)mix_plan(jobs[i], p);  // planned once already: cannot fail now
        if (int rc = mix_launch_direct(jobs[i], p.cfg, stream)) return rc;
        if (hook) {
            hook->job_stage[i] = sc.next++;
            if (int rc = hook->stage(hook->arg, stream)) return rc;
        }
    }
    if (done_event) e = hipEventRecord(done_event, stream);
    return fail_hip(e, "mixed launch");
}

int mix_launch_direct(const ppx_job &j, const ppx_config &c, hipStream_t s) {
    switch (j.op) {
        case PPX_OP_FFT: return fft_batched(j.in, j.out, j.n, j.batch, j.direction, &c, s);
        case PPX_OP_SCAN:
            return j.algo == PPX_JOB_SCAN_EXCLUSIVE ? scan_exclusive_batched(j.in, j.out, j.n, j.batch, j.dtype, &c, s)
                                                    : scan_batched(j.in, j.out, j.n, j.batch, j.dtype, &c, s);
        default: return tridiag_batched(j.in, j.b, j.c, j.d, j.out, j.n, j.batch, j.dtype, &c, s);
    }
}

// ------------------------------------------------ the allocation-free launch
// The same launch for callers that cannot allocate (code under graph capture,
// tight serving loops).  A small launch passes its records in the kernel
// arguments as launch_mixed does; any other keeps its tables in `scratch`, a file-scope device
// array holding at most kNoAllocJobs jobs and kNoAllocTiles tiles, whose
// address on each device is taken once at set-up (hipGetSymbolAddress; in
// host code the array's name is not a device address).  The table reaches the
// device through the kernel arguments of a few copy launches (the runtime
// copies kernel arguments when a launch is enqueued), so no host buffer
// outlives the call and no copy is issued from host memory; the tile
// counters are part of that table and start at zero with it.  Every call on
// a device shares its array: calls that overlap on one device race.
constexpr int kNoAllocJobs = PPX_NOALLOC_MAX_JOBS;
constexpr int kNoAllocTiles = PPX_NOALLOC_MAX_TILES;
constexpr int64_t kNoAllocBytes = mix_table_bytes(kNoAllocJobs, kNoAllocTiles) + 16;
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kTableChunk = 2048;  // table bytes per copy launch
struct TableChunk {
    unsigned offset, bytes;
    unsigned char data[kTableChunk];
};

__global__ __launch_bounds__(256) void k_mix_table_copy(char *tables, TableChunk c) {
    for (unsigned i = threadIdx.x; i < c.bytes; i += blockDim.x) tables[c.offset + i] = (char)c.data[i];
}

namespace {
std::mutex g_noalloc_mu;
std::vector<char *> g_scratch;  // per device ordinal: the array's device address
}  // namespace

// Set-up of the current device for the allocation-free launch: the device
// state and twiddle tables (static arrays), the family kernels' occupancy,
// and the address of `scratch` on this device.
static char *noalloc_scratch() {
    const DeviceInfo *di = device_info();
    if (!di) return nullptr;
    if (mix_prepare_kernels() != PPX_OK) return nullptr;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if ((int)g_scratch.size() <= di->device) g_scratch.resize(di->device + 1, nullptr);
    if (!g_scratch[di->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fail_hip(e == hipSuccess ? hipErrorInvalidSymbol : e, "scratch address");
            return nullptr;
        }
        g_scratch[di->device] = static_cast<char *>(p);
    }
    return g_scratch[di->device];
}

int launch_mixed_noalloc_impl(const ppx_job *jobs, int njobs, hipStream_t stream) {
    if (!jobs || njobs < 1) return fail(PPX_EINVAL, "no jobs");
    if (njobs > kNoAllocJobs)
        return fail(PPX_EINVAL, "launch_mixed_noalloc takes at most PPX_NOALLOC_MAX_JOBS (256) jobs");
    // header and job records, built on the stack
    alignas(16) char table[kMixHeaderBytes + sizeof(MixJob) * kNoAllocJobs];
    int64_t ntiles = 0;
    int direct[kNoAllocJobs], ndirect = 0;
    const int mask = mix_build_tables(jobs, njobs, table, &ntiles, direct, &ndirect);
    if (mask < 0) return mask;
    if (ntiles > kNoAllocTiles)
        return fail(PPX_EINVAL, "launch_mixed_noalloc takes at most PPX_NOALLOC_MAX_TILES (262144) tiles");
    char *d = noalloc_scratch();
    if (!d) return PPX_EDEVICE;
    const float2 *tw = static_cast<const float2 *>(device_info()->twiddles);
    int order[kMixFamilies];
    const int norder = mix_family_order(table, mask, order);
    if (mask && mix_args_fit(table, mask)) {  // a small launch: the records go in the kernel arguments
        if (int rc = mix_enqueue_args(table, mask, order, norder, tw, stream)) return rc;
    } else if (mask) {
        const MixHeader *h = reinterpret_cast<const MixHeader *>(table);
        const unsigned bytes = (unsigned)(kMixHeaderBytes + sizeof(MixJob) * (size_t)h->njobs);
        TableChunk c;
        for (unsigned off = 0; off < bytes; off += kTableChunk) {
            c.offset = off;
            c.bytes = std::min<unsigned>(kTableChunk, bytes - off);
            std::memcpy(c.data, table + off, c.bytes);
            hipLaunchKernelGGL(k_mix_table_copy, dim3(1), dim3(256), 0, stream, d, c);
            if (int rc = fail_hip(hipGetLastError(), "table copy")) return rc;
        }
        int64_t fam_tiles[kMixFamilies];
        for (int f = 0; f < kMixFamilies; ++f) fam_tiles[f] = h->ntiles[f];
        if (int rc = mix_enqueue(d, mask, fam_tiles, h->block, order, norder, tw, stream)) return rc;
    }
    for (int k = 0; k < ndirect; ++k) {  // jobs that fill the GPU alone: their tuned single calls
        MixPlan p;
        (void)mix_plan(jobs[direct[k]], p);
        if (int rc = mix_launch_direct(jobs[direct[k]], p.cfg, stream)) return rc;
    }
    return PPX_OK;
}

}  // namespace ppx

extern "C" int launch_mixed_noalloc(const ppx_job *jobs, int njobs, void *stream) {
    ppx::fail(PPX_OK, "");
    return ppx::launch_mixed_noalloc_impl(jobs, njobs, static_cast<hipStream_t>(stream));
}

extern "C" int launch_mixed(const ppx_job *jobs, int njobs, void *stream) {
    ppx::fail(PPX_OK, "");
    return ppx::launch_mixed_impl(jobs, njobs, static_cast<hipStream_t>(stream), nullptr);
}

extern "C" int ppx_mixed_families_complete(void) {
    for (int f = 0; f < ppx::kMixFamilies; ++f)
        if (!ppx::mix_kernel(f, false) || !ppx::mix_kernel(f, true)) return ppx::fail(PPX_EINVAL, "mixed launch: no kernel for family " + std::to_string(f));
    return PPX_OK;
}

extern "C" int ppx_mixed_argument_launch(const ppx_job *jobs, int njobs) {
    ppx::fail(PPX_OK, "");
    if (!jobs || njobs < 1) return ppx::fail(PPX_EINVAL, "no jobs");
    if (njobs > ppx::kMixMaxJobs) return ppx::fail(PPX_EINVAL, "too many jobs for one mixed launch");
    std::vector<char> table((size_t)ppx::mix_table_bytes(njobs, 0));
    std::vector<int> direct(njobs);
    int64_t ntiles = 0;
    int ndirect = 0;
    const int mask = ppx::mix_build_tables(jobs, njobs, table.data(), &ntiles, direct.data(), &ndirect);
    if (mask < 0) return mask;
    return ppx::mix_args_fit(table.data(), mask) ? 1 : 0;
}

extern "C" int ppx_mixed_tile_config(const ppx_job *job, ppx_config *cfg) {
    ppx::fail(PPX_OK, "");
    if (!job) return ppx::fail(PPX_EINVAL, "null job");
    ppx::MixPlan m;
    if (int rc = ppx::check_job(*job, &m)) return rc;
    if (cfg) *cfg = m.cfg;
    return m.per_tile;
}
