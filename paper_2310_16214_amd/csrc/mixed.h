// Mixed batched launch: the device-side tables and the kernel families.
//
// A mixed launch takes jobs of different operations, sizes and batch counts.
// Each job's problems are cut into tiles; a tile is what one workgroup of
// the job's kernel family processes at once, and its shape is the tuned
// single-call configuration of the job (the tune cache's entry for (op,
// dtype, n), else the analytical model's choice): the same radix, values per
// thread and exchange algorithm, with the problems per workgroup scaled from
// the tuned block size to the family's.  Those are the quantities a
// problem's arithmetic depends on, so every job computes the same values as
// the single call with that configuration.
//
// Families group the tile shapes by block size and register demand, because
// a kernel's VGPR count and LDS size are the maxima over the code it
// contains and set its occupancy for every tile it runs:
//   FFT, T = n/P <= 256 threads per problem: 256-thread workgroups;
//   FFT, T > 256: 1024-thread workgroups;
//   scan, likewise by T;
//   tridiagonal inside a wave (n/P <= 64), float32 / float64, each in a
//   light and a heavy register tier (mix_triw_family);
//   tridiagonal through LDS (CR and PCR of larger systems);
//   the CR -> PCR hybrid of systems spanning several waves.
// Each family has two kernels running its tiles: one whose jobs come in the
// kernel arguments, a workgroup per tile, for launches with few jobs per
// family; and a persistent one pulling tile indices from the family's
// counter until its tiles are drained, after a table expansion on the same
// stream.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ppx_internal.h"

namespace ppx {

enum MixFamily : int {
    kFamFft256 = 0,
    kFamFft1024,   // P = 16
    kFamFft1024P8, // P = 8: half the LDS and fewer registers, two workgroups per CU
    kFamScan256,
    kFamScan1024,
    kFamTriW32,    // in-wave, float32: CR, WM, LF with P <= 8
    kFamTriW32H,   // in-wave, float32: P = 16, and the PCR variants
    kFamTriW64,    // in-wave, float64, P <= 8
    kFamTriW64H,   // in-wave, float64, P = 16
    kFamTriLds,    // LDS CR / PCR, float32 and float64
    kFamTriBlk32,  // the CR -> PCR hybrid across waves, float32, P <= 8
    kFamTriBlk32H, // the same, float32, P = 16
    kFamTriBlk64,  // the same, float64, P <= 8
    kFamTriBlk64H, // the same, float64, P = 16 (512-thread workgroups)
    kMixFamilies
};

// One job as the kernels see it (72 bytes).
struct MixJob {
    int shape;            // family-specific code of the tile's kernel instantiation
    int flags;            // FFT: 1 = inverse; scan: 1 = exclusive
    int log2n;
    int per_tile;         // problems per tile
    long long batch;
    unsigned first_tile;  // index of the job's first tile in its family's list
    int family;
    const void *p[4];     // FFT / scan input; tridiagonal a, b, c, d
    void *out;            // FFT / scan output; tridiagonal x
};
static_assert(sizeof(MixJob) == 72, "job record layout");

// Header of a launch's tables; the jobs follow at byte kMixHeaderBytes, the
// tile lists (one 32-bit job index per tile, family after family) at
// tiles_off.
struct MixHeader {
    unsigned next[kMixFamilies];      // tile counters (0 at launch)
    unsigned ntiles[kMixFamilies];    // tiles per family
    unsigned tile_base[kMixFamilies]; // first entry of each family's list
    unsigned block[kMixFamilies];     // workgroup size of each family's tiles (host use)
    unsigned njobs;
    unsigned tiles_off;               // byte offset of the tile lists
};
constexpr int kMixHeaderBytes = 256;
static_assert(sizeof(MixHeader) <= kMixHeaderBytes, "header layout");

constexpr int kMixMaxJobs = 1 << 14;
constexpr int kMixMaxTiles = 1 << 20;

// Bytes of the tables of a launch with njobs jobs and ntiles tiles.
constexpr int64_t mix_table_bytes(int64_t njobs, int64_t ntiles) {
    return kMixHeaderBytes + njobs * (int64_t)sizeof(MixJob) + ntiles * 4;
}

// ---- shape codes
// FFT (radix = P in {4, 8, 16}): ((log2n * 3 + pidx) * 2 + split).
constexpr int fft_pidx(int P) { return P == 4 ? 0 : P == 8 ? 1 : 2; }
constexpr int mix_fft_shape(int log2n, int P, bool split) { return (log2n * 3 + fft_pidx(P)) * 2 + (split ? 1 : 0); }
constexpr int kMixFftShapes = (kFftLog2NMax + 1) * 6;
// Scan: ((dtype * 5 + log2(P) - 1) * 2 + lf) with dtype PPX_I32/F32/F64.
constexpr int mix_scan_shape(int dtype, int lp, bool lf) { return (dtype * 5 + lp - 1) * 2 + (lf ? 1 : 0); }
constexpr int kMixScanShapes = 3 * 5 * 2;
// In-wave tridiagonal: (variant - PPX_TRI_CR_PCR) * 4 + log2(P) - 1 (the
// in-wave variants are the codes PPX_TRI_CR_PCR .. PPX_TRI_LF).
constexpr int mix_triw_shape(int base, int lp) { return (base - PPX_TRI_CR_PCR) * 4 + lp - 1; }
constexpr int kMixTriwShapes = (PPX_TRI_LF - PPX_TRI_CR_PCR + 1) * 4;
// Family of an in-wave tridiagonal shape (variant without the persistent
// flag, P).
constexpr int mix_triw_family(bool f64, int algo, int P) {
    return f64 ? (P == 16 ? kFamTriW64H : kFamTriW64)
               : (P == 16 || algo == PPX_TRI_PCR_SHFL || algo == PPX_TRI_PCR_REG ? kFamTriW32H : kFamTriW32);
}
// LDS tridiagonal: dtype_is_f64 * 2 + (algo == PPX_TRI_PCR).
constexpr int mix_tril_shape(bool f64, bool pcr) { return (f64 ? 2 : 0) + (pcr ? 1 : 0); }

// Block size and dynamic LDS bytes of each family's kernel.
constexpr int mix_block(int fam) {
    return fam == kFamFft1024 || fam == kFamFft1024P8 || fam == kFamScan1024 || fam == kFamTriLds ||
                   fam == kFamTriBlk32 || fam == kFamTriBlk32H || fam == kFamTriBlk64
               ? 1024
           : fam == kFamTriBlk64H ? 512
                                  : 256;
}
constexpr int kMixTriLdsBudget = 128 * 1024;
int64_t mix_lds_bytes(int fam);

// What a family kernel is launched with.  A launch in which every family
// has at most kMixArgJobs jobs passes each family's job records here
// (first_tile counted within the family) to the family's argument kernel,
// whose workgroup b runs tile b: no table in device memory, no expansion, no
// counter, one launch per family.  Any other launch passes the device tables
// (tables) to the persistent kernels, which claim tiles from the counters.
constexpr int kMixArgJobs = PPX_MIXED_ARG_JOBS;
struct MixArgs {
    const char *tables;  // persistent kernels: the device tables
    unsigned ntiles;     // argument kernels: the family's tiles
    unsigned njobs;      // argument kernels: records in jobs[]
    MixJob jobs[kMixArgJobs];
};
static_assert(sizeof(MixArgs) <= 4096 - 64, "kernel arguments are limited to 4 KiB");

// Kernel of a family (signature mix_kernel_t), persistent or taking its
// records in the arguments, from the translation unit that instantiates it.
typedef void (*mix_kernel_t)(MixArgs a, const float2 *tw);
const void *mix_fft_kernel(int fam, bool args);
const void *mix_scan_kernel(int fam, bool args);
const void *mix_tri_kernel(int fam, bool args);
// Writes every family's tile list from the job records (one launch).
const void *mix_expand_kernel();
constexpr int kMixExpandBlocks = 512;
constexpr int kMixExpandThreads = 256;

// ---- host side (fused.hip)
// How a job is cut into tiles: its family, the kernel shape code, problems
// per tile, flags, tile count, and the single-call configuration whose
// arithmetic the tiles follow (the tuned one with the persistent flag
// cleared; a radix = P substitute where the tuned FFT shape is not one the
// families hold).
// A job that by itself fills the GPU and whose tuned configuration is a
// persistent variant (which prefetches the next group while computing the
// current one, something a tile of the shared loop cannot do) runs as its
// own single call with that configuration instead (direct = true, no tiles).
// A tile's workgroup size (block) is the tuned one (threads_per_block), kept
// within what the family's kernel allows (mix_block) and at least a wave and
// a problem's threads (tpp); the problems per tile are block / tpp, so a job
// alone runs tiles of exactly its tuned shape (G_b problems of P values per
// thread in L threads).  A launch runs each family at the largest block of
// its jobs.  LDS-exchange tridiagonal tiles (tpp = 0) are sized by LDS.
struct MixPlan {
    int family, shape, per_tile, flags;
    int tpp, block;
    int64_t ntiles;
    ppx_config cfg;
    bool direct;
};
// The single-call configuration of a job with cfg == NULL (tridiagonal: the
// job's family).
int job_config(const ppx_job &j, ppx_config &c);
int mix_plan(const ppx_job &j, MixPlan &m);
// Plans every job and writes the header and job records into buf; returns
// the mask of families with tiles or a negative error.
// Direct jobs get no record; their indices go to direct[0 .. *ndirect)
// (room for njobs entries).  rec_job (optional, njobs entries) receives the
// job index of each record.
int mix_build_tables(const ppx_job *jobs, int njobs, char *buf, int64_t *ntiles_out, int *direct, int *ndirect,
                     int *rec_job = nullptr);
// The families of `mask` in launch order: ascending total elements of
// their jobs, so that the families of small jobs finish first.  Returns
// their count.
int mix_family_order(const char *table, int mask, int *order);
// Called after each family kernel is enqueued (may be empty).
typedef int (*mix_after_family_t)(void *arg, int fam, hipStream_t s);
// Launches job j alone with configuration c (a direct job).
int mix_launch_direct(const ppx_job &j, const ppx_config &c, hipStream_t s);
// Occupancy of every family kernel on the current device (once).
int mix_prepare_kernels();
// Expansion plus the family kernels of `mask` in the given order, on stream
// s, in workgroups of blocks[f] threads, each grid capped at the family's
// tile count ntiles[f].
int mix_enqueue(char *d_tables, int mask, const int64_t *ntiles, const unsigned *blocks, const int *order, int norder,
                const float2 *tw, hipStream_t s, mix_after_family_t after = nullptr, void *arg = nullptr);
// Whether the launch planned in `table` (header and records) can pass its
// jobs as kernel arguments (at most kMixArgJobs per family), and if so its
// launches: one argument kernel per family in mask, a workgroup per tile.
// A launch too small to fill the GPU runs smaller workgroups (fewer
// problems per tile, never fewer threads than a problem or a wave needs).
bool mix_args_fit(const char *table, int mask);
int mix_enqueue_args(const char *table, int mask, const int *order, int norder, const float2 *tw, hipStream_t s,
                     mix_after_family_t after = nullptr, void *arg = nullptr);

// ---- the tile loop shared by the families
// ARGS: the records come in the kernel arguments and workgroup b runs tile b
// (the grid is the family's tile count), its job found by a scan of the
// family's few records, read through the constant address space (the
// launch's explicit arguments start the kernarg segment, MixArgs first).
// Otherwise the kernel is persistent: it claims tile indices of family FAM
// from its counter in the device tables until they run out, the next index
// being claimed while the current tile is processed, and looks the job up
// in the family's tile list.
// Either way body(job, first problem, problem count, tx, nt) runs each tile,
// nt being the workgroup's size (the tuned one, at most mix_block(FAM); see
// MixPlan) and tx the thread's
// index in the workgroup passed through an empty asm that
// claims to change it: without it the compiler hoists every address derived
// from the thread index out of the loop, for every shape a family holds, and
// keeps them all live (the FFT families then spilled).  Every thread of the
// workgroup runs the same iterations, so all reach every barrier.
typedef const __attribute__((address_space(4))) MixJob *mix_arg_job_ptr;

__device__ __forceinline__ MixJob mix_load_job(mix_arg_job_ptr r) {
    MixJob j;
    j.shape = r->shape;
    j.flags = r->flags;
    j.log2n = r->log2n;
    j.per_tile = r->per_tile;
    j.batch = r->batch;
    j.first_tile = r->first_tile;
    j.family = r->family;
    for (int i = 0; i < 4; ++i) j.p[i] = r->p[i];
    j.out = r->out;
    return j;
}

template <typename Body>
__device__ __forceinline__ void mix_run_tile(const MixJob &j, unsigned t, int nt, Body &body) {
    const long long first = (long long)(t - j.first_tile) * j.per_tile;
    const int count = (int)min((long long)j.per_tile, j.batch - first);
    int tx = threadIdx.x;
    asm volatile("" : "+v"(tx));
    body(j, first, count, tx, nt);
}

template <int FAM, bool ARGS, typename Body>
__device__ __forceinline__ void mix_tile_loop(const MixArgs &a, Body &&body) {
    if constexpr (ARGS) {
        const mix_arg_job_ptr recs = reinterpret_cast<mix_arg_job_ptr>(
            (const __attribute__((address_space(4))) char *)__builtin_amdgcn_kernarg_segment_ptr() +
            offsetof(MixArgs, jobs));
        const unsigned t = blockIdx.x;
        unsigned k = 0;
        while (k + 1 < a.njobs && recs[k + 1].first_tile <= t) ++k;
        mix_run_tile(mix_load_job(recs + k), t, (int)blockDim.x, body);
    } else {
        __shared__ unsigned s_tile;
        const MixHeader *h = reinterpret_cast<const MixHeader *>(a.tables);
        const MixJob *jobs = reinterpret_cast<const MixJob *>(a.tables + kMixHeaderBytes);
        const unsigned *tiles = reinterpret_cast<const unsigned *>(a.tables + h->tiles_off) + h->tile_base[FAM];
        unsigned *ctr = const_cast<unsigned *>(&h->next[FAM]);
        const unsigned ntiles = h->ntiles[FAM];
        if (threadIdx.x == 0) s_tile = atomicAdd(ctr, 1u);
        __syncthreads();
        unsigned t = __builtin_amdgcn_readfirstlane(s_tile);
        while (t < ntiles) {
            unsigned next = 0;
            if (threadIdx.x == 0) next = atomicAdd(ctr, 1u);
            mix_run_tile(jobs[__builtin_amdgcn_readfirstlane(tiles[t])], t, (int)blockDim.x, body);
            __syncthreads();  // every thread is done with s_tile and the tile's LDS
            if (threadIdx.x == 0) s_tile = next;
            __syncthreads();
            t = __builtin_amdgcn_readfirstlane(s_tile);
        }
    }
}

}  // namespace ppx
