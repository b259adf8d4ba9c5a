// Large-N batched FFT (2^14 < n <= 2^23) in two passes of column FFTs -- the
// multi-kernel decomposition of Sec. IV-A for sizes beyond one workgroup.
//
// With n = n1 * n2 and input index j = j1 + n1 * j2 (j1 < n1, j2 < n2), the
// output index k = k2 + n2 * k1 factors the transform as
//     X[k2 + n2 k1] = sum_j1 w_n1^{j1 k1} w_n^{j1 k2} sum_j2 x[j1 + n1 j2] w_n2^{j2 k2}.
// Pass A views x as n2 rows of n1 columns and transforms every column (length
// n2), multiplies element (j1, k2) by w_n^{j1 k2} and writes column j1 as row
// j1 of Z (n1 rows of n2 values).  Pass B transforms every column of Z
// (length n1) in place; column k2, element k1 is then X[k2 + n2 k1] exactly
// where it lies.  So the output buffer holds Z and no workspace is needed,
// but the input must be a different buffer.
//
// A workgroup takes a tile of TC adjacent columns (a plan parameter per
// pass): it reads them row by row (TC lanes on TC consecutive values) into
// LDS, transforms the TC columns with the single-pass stage code (radix
// R = P, T = len/P threads per column, exchanges in LDS), and writes the tile
// back the same way (pass B) or row by row (pass A, 512-byte runs per wave).
// The LDS layout (TileLayout) spreads a row access over the banks and keeps
// the exchanges of long columns aligned to the stage swizzles.  Tiles of 16, 32 or 64
// columns read and write runs of 128 to 512 bytes; tiles of 2, 4 or 8 (runs
// of 16 to 64 bytes) are the only ones that fit LDS for columns of 2048 to
// 8192 values (pass A, with its tables, up to 4096), and are also valid for
// shorter columns, where they give more workgroups.  Narrow tiles number the
// workgroups so that the tiles sharing a row's cache lines run on one XCD,
// whose L2 then serves the lines to all of them, and the workgroups in flight
// together cover whole stretches of the rows (tile_order).  Tiles that leave
// room for one workgroup per CU run persistent, loading the next tile while
// transforming the current one.
//
// The pass-A twiddles w_n^m (m < n <= 2^23) are the product of three table
// entries, w_{2^23}^{q mod 2^10} * w_{2^13}^{(q div 2^10) mod 2^10} *
// w_8^{q div 2^20} with q = m * 2^23 / n: 1024 + 1024 + 8 values built on the
// host in double precision, copied into LDS by every pass-A workgroup.
#include "fft_device.h"

#include <algorithm>
#include <map>
#include <mutex>

namespace ppx {

// LDS layout of a tile: element e of column c at swz_c(poff(c) + (e ^ px(c))).
// The row accesses (the tile's loads, pass B's stores) put TC columns x
// 64 / TC consecutive rows in a wave; the stage exchanges put T = len / R
// consecutive threads of a column in a wave.
// * T >= 64 (one column per wave in the exchanges): columns at multiples of
//   len, so each column is aligned to the 256-value blocks of the stage
//   swizzles and its exchanges are as conflict-free as a single-pass
//   transform's.  The LDS serves 16 lanes of 8-byte words together; in a row
//   access those are 16 / TC consecutive rows of each of TC columns (TC <=
//   16) or one row of 16 columns.  px(c) = c * max(1, 16 / TC) (mod 16) puts
//   each column's run on its own banks, so the 16 words fall on 16 banks.
//   It is below 16 and the index constants of the accesses are multiples of
//   64, so the XOR commutes with them and they stay instruction offsets.
// * T < 64 (several columns per wave): columns padded to len + 1 values, so
//   that the columns of a wave fall on different banks; px = 0.
template <int R, int LOG2LEN, int TC>
struct TileLayout {
    static constexpr int len = 1 << LOG2LEN;
    static constexpr bool kAligned = LOG2LEN - clog2(R) >= 6;
    __device__ __forceinline__ static int poff(int c) { return kAligned ? c * len : c * (len + 1); }
    __device__ __forceinline__ static int px(int c) { return kAligned ? (c * (TC < 16 ? 16 / TC : 1)) & 15 : 0; }
    __device__ __forceinline__ static int slot(int c, int e) { return swz_c(poff(c) + (e ^ px(c))); }
    // slot(c, e + k) for e < 2^m and k a multiple of 2^m, m >= 6 (with
    // T < 64: any e, k).  e + k then has k's bits and e's bits apart, and so
    // have poff(c) (a multiple of len) and e ^ px(c): the swizzle of the sum is
    // that of poff(c) + (e ^ px(c)), XORed with k's swizzle term (bits 4..7 of
    // k, moved to 0..3), plus k.  Written this way, one base per thread serves
    // every k, and constant k become instruction offsets.
    __device__ __forceinline__ static int slot_k(int c, int e, int k) {
        if constexpr (kAligned) return (swz_c(poff(c) + (e ^ px(c))) ^ ((k >> 4) & 15)) + k;
        else return swz_c(poff(c) + e + k);
    }
};

__device__ __forceinline__ int tw_swz(int j) { return j ^ ((j >> 5) & 31); }

constexpr int kTwLargeVals = 1024 + 1024 + 8;  // the three pass-A tables
// Shortest run of a pass-B row store (bytes) that goes out non-temporal: a
// whole cache line.  Shorter runs are partial lines, which non-temporal
// stores send to memory one by one instead of merging them in L2 with the
// neighbouring tiles' parts (measured: 11-15% slower calls with 2- and
// 4-column tiles, no gain with 8).
constexpr int kTileNtRun = 128;
constexpr int kLog2NLargeMax = 23;

// float2 slots of a tile: TC padded columns, rounded up to whole 256-value
// blocks (the swizzle permutes within aligned blocks of 256)
__host__ __device__ constexpr int tile_vals(int log2len, int tc) { return (tc * ((1 << log2len) + 1) + 255) / 256 * 256; }

// Workgroups whose tile (and, in pass A, tables) take more than half of the
// LDS run one per CU; such tile shapes are launched persistent
// (k_fft_tile_p), so that a CU's loads overlap its own stages.  In pass B
// only for columns of 1024 values or more (the aligned tile layout, whose
// accesses are a base register plus offsets): the persistent pass B on
// shorter, wider tiles needs more than the 128 registers of a 1024-thread
// workgroup.
__host__ __device__ constexpr bool tile_persistent(int log2len, int tc, bool pass_a) {
    return (pass_a || log2len >= 10) &&
           ((int64_t)tile_vals(log2len, tc) + (pass_a ? kTwLargeVals : 0)) * (int64_t)sizeof(float2) > 80 * 1024;
}

// Tile order.  Workgroups are dealt to the 8 XCDs in turn (XCD = workgroup
// index mod 8), each with its own L2.  The LG = 16 / TC adjacent tiles that
// share a row's 128-byte lines (TC < 16) go to one XCD, so each line is
// fetched into one L2 and served from there to all of them; and each run of
// 8 * LG consecutive workgroups takes 8 * LG consecutive tiles, so the
// workgroups in flight together cover whole stretches of every row they
// read (rather than each XCD walking its own eighth of the tiles: 4-10%
// faster calls from 2^19 to 2^23).  A permutation of [0, 8 * LG * k).
template <int TC>
__device__ __forceinline__ long long tile_order(long long b) {
    constexpr int LG = TC < 16 ? 16 / TC : 1;
    const long long x = b & 7, w = b >> 3;
    return (w / LG) * (8 * LG) + LG * x + (w % LG);
}

// Step order of the persistent tiles.  At each step the grid (G workgroups)
// covers G consecutive positions of its walk; where a problem's row holds
// m = tiles / G >= 2 times that many tiles (long rows), consecutive steps
// would each read one m-th of every row, in one stretch.  Instead, the m
// steps over a row's tiles take its line groups (the LG = 16 / TC tiles
// sharing 128-byte lines) in turn, step h the groups h, h + m, h + 2m, ...,
// so every step reads lines spread over whole rows (6% faster calls at
// 2^23, where both passes' rows hold 2 G tiles).  A workgroup whose walk
// starts at position t0 < G (group g0 = t0 / LG, lane i0 = t0 mod LG) then
// takes tiles (g0 m + h) LG + i0 of row r at step r m + h: from one tile to
// the next it adds LG, or LG + tiles - m LG where h wraps; no division in
// the loop.
// The walk is a separate instantiation (WALK), launched where a row holds
// 2 G tiles or more (tile_walk_reorders); elsewhere the identity walk keeps
// the kernel's code as it was (the walk's state, carried through the loop,
// measured 3.6% slower at 2^22 even where it changes no tile).
__host__ __device__ constexpr int tile_line_group(int tc) { return tc < 16 ? 16 / tc : 1; }
inline bool tile_walk_reorders(long long G, long long tiles, int tc) {
    return tiles >= 2 * G && tiles % G == 0 && G % tile_line_group(tc) == 0;
}
template <int TC>
struct TileWalk {
    static constexpr int LG = tile_line_group(TC);
    long long m, wrap;
    __device__ __forceinline__ TileWalk(long long G, long long tiles) : m(tiles / G), wrap(tiles - (tiles / G - 1) * LG) {}
    __device__ __forceinline__ long long first(long long t0) const { return (t0 / LG) * m * LG + t0 % LG; }
    __device__ __forceinline__ long long next(long long tile, int h) const { return tile + (h + 1 < m ? LG : wrap); }
    __device__ __forceinline__ int next_h(int h) const { return h + 1 < m ? h + 1 : 0; }
};

// float2 entries of a column transform's stage twiddle bases (every stage but
// the first: w^k, w^{4k} and, radix 16, w^{8k} for k below the stage's span),
// which the persistent tiles keep in LDS (after the tables in pass A).
__host__ __device__ constexpr int tile_stage_tw_vals(int radix, int log2len) {
    const int lr = radix == 16 ? 4 : 3;
    const int nst = (log2len + lr - 1) / lr;
    const int first = log2len % lr ? log2len % lr : lr;
    int e = 0;
    for (int i = 0; i < nst - 1; ++i) e += (radix == 16 ? 3 : 2) << (first + i * lr);
    return e;
}

// Pass A: the three twiddle tables into LDS after the tile.  Read from global
// memory in the store loop, each table read would wait for the stores issued
// before it (vector memory operations complete in issue order).  The lanes
// of the store loop read the low table at a stride of (column index) * 2^23 /
// n entries, often a multiple of 32; the two large tables are stored
// XOR-swizzled (bits 5..9 into 0..4) so that such strides spread over the
// banks.
__device__ __forceinline__ void tile_tables_to_lds(float2 *tlo, float2 *thi, float2 *tht, const float2 *__restrict__ tw_lo,
                                                   const float2 *__restrict__ tw_hi) {
    for (int j = threadIdx.x; j < 1024; j += blockDim.x) {
        tlo[tw_swz(j)] = tw_lo[j];
        thi[tw_swz(j)] = tw_hi[j];
    }
    if (threadIdx.x < 8) tht[threadIdx.x] = tw_hi[1024 + threadIdx.x];
}

// The stages of a tile's columns with the twiddle bases read from LDS (twl,
// laid out by fft_tw_to_lds), the form the persistent pass A uses: the stage
// code of the single-pass kernels reads them from global memory, and such a
// read, issued after the next tile's loads, waits for those loads too
// (vector memory operations complete in issue order).  Radix R = P: one
// butterfly per thread and stage after a first stage of the remaining bits.
// The last stage leaves its results in LDS at their output positions (XORed
// with pxor, then swizzled: pxor < 64 <= T, and the last stage's span is at
// least 64, so XORing the thread index does the same).
template <int R, int LOG2LEN, int LNS, int IDX, typename Hook>
__device__ __forceinline__ void tile_stages_twl(float2 (&v)[R], float2 *buf, int poff, int pxor, int tid,
                                                const float2 *twl, const Hook &hook) {
    constexpr int P = R;
    constexpr int REM = LOG2LEN % clog2(R);
    constexpr int RS = (LNS == 0 && REM != 0) ? (1 << REM) : R;
    constexpr int LRS = clog2(RS);
    constexpr int T = 1 << (LOG2LEN - clog2(P));
    if constexpr (LNS == 0) {
        stage_butterflies<RS, P, true>(v, tid, T, 0, nullptr);
    } else {
        constexpr int OFF = fft_tw_offset<R, LOG2LEN>(IDX);
        const int k = tid & ((1 << LNS) - 1);
        TwBase b;
        b.w1 = twl[OFF + k];
        if constexpr (RS >= 8) b.w4 = twl[OFF + (1 << LNS) + k];
        if constexpr (RS >= 16) b.w8 = twl[OFF + (2 << LNS) + k];
        float2 w[RS];
        stage_twiddles_from<RS>(w, b);
#pragma unroll
        for (int q = 1; q < RS; ++q) v[q] = cmul(v[q], w[q]);
        RegDFT<RS>::run(v);
    }
    if constexpr (LNS + LRS == LOG2LEN) {
        static_assert(P == RS, "the last stage is a full radix-R stage, one butterfly per thread");
        if constexpr (LNS >= 6) {
            // aligned layout (T = 2^LNS >= 64): output position (tid ^ pxor) + q T,
            // swizzled as in TileLayout::slot_k
            const int b = swz_c(poff + (tid ^ pxor));
#pragma unroll
            for (int q = 0; q < RS; ++q) buf[(b ^ (((q << LNS) >> 4) & 15)) + (q << LNS)] = v[q];
        } else {
#pragma unroll
            for (int q = 0; q < RS; ++q) buf[swz_c(poff + stage_out_pos<RS>(tid ^ pxor, LNS, q))] = v[q];
        }
    } else {
        stage_exchange<RS, P, false>(v, buf, poff, tid, T, LNS);
        constexpr int S = LNS == 0 ? 0 : 1 + (LNS - (REM ? REM : clog2(R))) / clog2(R);
        hook.template at<S>();
        tile_stages_twl<R, LOG2LEN, LNS + LRS, LNS == 0 ? IDX : IDX + 1, Hook>(v, buf, poff, pxor, tid, twl, hook);
    }
}

// The tile in LDS (written by the caller, no barrier yet): transform its TC
// columns and write them out.  NT = len * TC / R threads; tx is the thread's
// index in the workgroup.  PERSIST (pass A only) takes the stage twiddle
// bases from LDS (tw then points there) and stores through a descriptor of
// the problem's output, with the column step in the scalar operand.
template <int R, int LOG2LEN, bool PASS_A, int TC, bool PERSIST, typename Hook = NoStageHook>
__device__ __forceinline__ void tile_transform_store(float2 *buf, const float2 *tlo, const float2 *thi, const float2 *tht,
                                                     float2 *out, long long base, int c0, long long cols, int log2n,
                                                     float sgn, const float2 *__restrict__ tw, int tx,
                                                     const Hook &hook = Hook{}) {
    constexpr int len = 1 << LOG2LEN;
    constexpr int P = R;
    constexpr int lT = LOG2LEN - clog2(P);
    constexpr int T = 1 << lT;
    constexpr int LTC = clog2(TC);
    constexpr int NT = len * TC / R;
    using Lay = TileLayout<R, LOG2LEN, TC>;
    // the problem's n values of the output (offsets below 2^26 bytes)
    const __amdgpu_buffer_rsrc_t orsrc = __builtin_amdgcn_make_buffer_rsrc(
        out + base, (short)0, (int)((1LL << log2n) * (long long)sizeof(float2)), kBufferFlags);
    __syncthreads();
    const int lp = tx >> lT;  // column of the tile
    const int tid = tx & (T - 1);
    float2 v[P];
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = buf[Lay::slot_k(lp, tid, j * T)];
    __syncthreads();
    if constexpr (PASS_A) fft_conj<P>(v, sgn);  // the inverse: conjugated in pass A, out in pass B
    // the last stage's writes recompute their base from an opaque copy of
    // px, rather than keep the gather's bases live through the stages
    int pxl = Lay::px(lp);
    if constexpr (Lay::kAligned) asm volatile("" : "+v"(pxl));
    if constexpr (PERSIST)  // tw: the stage twiddle bases in LDS
        tile_stages_twl<R, LOG2LEN, 0, 0, Hook>(v, buf, Lay::poff(lp), pxl, tid, tw, hook);
    else
        fft_stages_ct<R, P, false, LOG2LEN, 0, true, Hook>(v, buf, Lay::poff(lp), nullptr, tid, true, sgn, tw, hook,
                                                           pxl);
    __syncthreads();
    if constexpr (PASS_A) {
        // Element (c, e) of the tile is stored at row c0 + c, position e, of
        // the intermediate, times w^{(c0 + c) e}; consecutive threads take
        // consecutive e (runs of 512 bytes per wave).  With TC >= R thread t
        // takes e = t mod len and the R columns ct + k * CS (ct = t div len,
        // CS = TC / R): its twiddles form a geometric sequence with ratio
        // w^{CS e}.  With TC < R it takes the R / TC rows e = t + r * NT and
        // all TC columns of each: one sequence of ratio w^e per row.
        // Sequences are started and stepped from the tables (at most R - 1
        // products, so a few ulp of drift at most).
        const int shift = kLog2NLargeMax - log2n;
        auto table_tw = [&](unsigned m) {  // w_n^m for m < n
            const unsigned q = m << shift;  // < 2^23
            return cmul(cmul(tlo[tw_swz((int)(q & 1023u))], thi[tw_swz((int)((q >> 10) & 1023u))]), tht[q >> 20]);
        };
        if constexpr (TC >= R) {
            constexpr int CS = TC / R;
            const int e = tx & (len - 1), ct = tx >> LOG2LEN;
            float2 w = table_tw((unsigned)(c0 + ct) * (unsigned)e);
            const float2 step = table_tw((unsigned)CS * (unsigned)e);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int c = ct + k * CS;
                const float2 y = cmul(buf[Lay::slot(c, e)], w);
                if constexpr (PERSIST)  // one vector offset, the column step in the scalar operand
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, y), orsrc,
                                                          ((c0 + ct) * len + e) * (int)sizeof(float2),
                                                          k * CS * len * (int)sizeof(float2), kStoreNT);
                else
                    store_nt_any(out + base + (long long)(c0 + c) * len + e, y);
                w = cmul(w, step);
            }
        } else {
#pragma unroll
            for (int r = 0; r < R / TC; ++r) {
                const int e = tx + r * NT;
                float2 w = table_tw((unsigned)c0 * (unsigned)e);
                const float2 step = table_tw((unsigned)e);
#pragma unroll
                for (int c = 0; c < TC; ++c) {
                    const float2 y = cmul(buf[Lay::slot_k(c, tx, r * NT)], w);
                    if constexpr (PERSIST)
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, y), orsrc,
                                                              (c0 * len + tx) * (int)sizeof(float2),
                                                              (c * len + r * NT) * (int)sizeof(float2), kStoreNT);
                    else
                        store_nt_any(out + base + (long long)(c0 + c) * len + e, y);
                    w = cmul(w, step);
                }
            }
        }
    } else if constexpr (PERSIST) {
        // element i = tx + k * NT: column tx mod TC, row tx div TC + k * T;
        // one vector offset, the row step in the scalar operand, and a
        // constant number of stores (the wait for the next tile's loads then
        // leaves these stores in flight)
        const int c = tx & (TC - 1), e0 = tx >> LTC;
        const int voff = (e0 * (int)cols + c0 + c) * (int)sizeof(float2);
        const int rstep = T * (int)cols * (int)sizeof(float2);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const float2 y = buf[Lay::slot_k(c, e0, k * T)];
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, make_float2(y.x, sgn * y.y)), orsrc, voff,
                                                  k * rstep, TC * (int)sizeof(float2) >= kTileNtRun ? kStoreNT : 0);
        }
    } else {
        for (int i = tx; i < len * TC; i += NT) {
            const int c = i & (TC - 1), e = i >> LTC;
            const float2 y = buf[Lay::slot(c, e)];
            if constexpr (TC * (int)sizeof(float2) >= kTileNtRun)
                store_nt_any(out + base + e * cols + c0 + c, make_float2(y.x, sgn * y.y));
            else
                out[base + e * cols + c0 + c] = make_float2(y.x, sgn * y.y);
        }
    }
}

// TC: columns per tile (2 to 64: runs of 16 to 512 bytes).  One workgroup
// per tile; `total` (the tiles of the batch) is unused.
template <int R, int LOG2LEN, bool PASS_A, int TC>
__global__ __launch_bounds__(1024) void k_fft_tile(const float2 *in, float2 *out, const float2 *__restrict__ tw,
                                                    const float2 *__restrict__ tw_lo,
                                                    const float2 *__restrict__ tw_hi, int log2n,
                                                    int log2cols, long long tiles, long long, float sgn) {
    constexpr int len = 1 << LOG2LEN;  // column length: the sub-transform size
    constexpr int LTC = clog2(TC);
    constexpr int NT = len * TC / R;
    extern __shared__ float4 lds_raw[];
    float2 *buf = reinterpret_cast<float2 *>(lds_raw);
    long long blk = blockIdx.x;
    if constexpr (TC < 16)
        if (gridDim.x % (8 * (16 / TC)) == 0) blk = tile_order<TC>(blk);
    const long long prob = blk / tiles;
    const int c0 = (int)(blk % tiles) * TC;
    const long long base = prob << log2n;
    const long long cols = 1LL << log2cols;
    float2 *tlo = buf + tile_vals(LOG2LEN, TC), *thi = tlo + 1024, *tht = thi + 1024;
    using Lay = TileLayout<R, LOG2LEN, TC>;
    if constexpr (PASS_A) tile_tables_to_lds(tlo, thi, tht, tw_lo, tw_hi);
    for (int i = threadIdx.x; i < len * TC; i += NT) {
        const int c = i & (TC - 1), e = i >> LTC;
        buf[Lay::slot(c, e)] = in[base + e * cols + c0 + c];
    }
    tile_transform_store<R, LOG2LEN, PASS_A, TC, false>(buf, tlo, thi, tht, out, base, c0, cols, log2n, sgn, tw,
                                                        (int)threadIdx.x);
}

// Buffer descriptor of tile t's rows (the problem from column c0 on); no
// records (loads return zero, no memory access) for t >= total.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const float2 *in, long long t, long long total,
                                                            long long tiles, int tc, int log2n) {
    const bool ok = t < total;
    const long long prob = ok ? t / tiles : 0;
    const int c0 = ok ? (int)(t % tiles) * tc : 0;
    const char *p = reinterpret_cast<const char *>(in + (prob << log2n) + c0);
    const int bytes = ok ? (int)(((1LL << log2n) - c0) * (long long)sizeof(float2)) : 0;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, bytes, kBufferFlags);
}

// The thread's R values of a tile's rows: element i = tx + k * NT, column
// i mod TC (= tx mod TC), row i div TC (= tx div TC + k * len / R).  Byte
// offsets stay below 2^26 (n <= 2^23 values).
// Chunk C of NC: the loads k with k * NC / R == C (the chunks partition them).
template <int R, int LOG2LEN, int TC, int C = 0, int NC = 1>
__device__ __forceinline__ void tile_load_rows(float2 (&pre)[R], __amdgpu_buffer_rsrc_t r, int cols, int tx) {
    constexpr int LTC = clog2(TC);
    const int voff = ((tx >> LTC) * cols + (tx & (TC - 1))) * (int)sizeof(float2);
    const int rstride = ((1 << LOG2LEN) / R) * cols * (int)sizeof(float2);
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (k * NC / R == C)
            pre[k] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, k * rstride, 0));
}

// The persistent pass A's next-tile loads, spread over the stages: chunk 0
// before the first stage, chunk s after the exchange that follows stage
// s - 1, NC = (stages - 1) chunks, so none is issued in the last stage, just
// before the stores.  (A burst of every load at the tile's start, on the
// heels of the previous tile's stores, leaves the memory system idle during
// the later stages.)
template <int R, int LOG2LEN, int TC>
struct TilePrefetch {
    static constexpr int NST = (LOG2LEN + clog2(R) - 1) / clog2(R);
    static constexpr int NC = NST > 2 ? NST - 1 : 1;
    float2 (&pre)[R];
    __amdgpu_buffer_rsrc_t r;
    int cols, tx;
    template <int S>
    __device__ __forceinline__ void at() const {
        if constexpr (S + 1 < NC) tile_load_rows<R, LOG2LEN, TC, S + 1, NC>(pre, r, cols, tx);
    }
};

// Persistent form for tiles that leave room for one workgroup per CU: a grid
// of at most one workgroup per CU walks the tiles and loads the next tile's
// values into registers while it transforms and stores the current one, so
// that a CU's loads overlap its own stages (one workgroup per CU otherwise
// alternates between loading and computing).  The loads go out in chunks
// between the stages (TilePrefetch), and the stages read their twiddle bases
// from LDS (tile_stages_twl), so no global read inside a tile waits for the
// prefetch.  The loads of a tile that does
// not exist go through a descriptor without records, so no branch surrounds
// them; the first tile is peeled, so the loop is entered only after a whole
// tile (loads, then stores), the same history as its back edge, and the
// compiler's wait before the LDS writes covers the prefetch only, not the
// stores issued after it.  Workgroup b walks positions tile_order(b) + k * G
// (G the grid; where G is a multiple of 8 * 16 / TC and divides the tile
// count, else b + k * G): at each step the grid covers G consecutive
// positions, and the tiles sharing a row's cache lines are in flight on one
// XCD together; TileWalk maps positions to tiles.  Every thread of a
// workgroup runs the same iterations, so all reach every barrier.
template <int R, int LOG2LEN, bool PASS_A, int TC, bool WALK = false>
__global__ __launch_bounds__(1024) void k_fft_tile_p(const float2 *in, float2 *out, const float2 *__restrict__ tw,
                                                      const float2 *__restrict__ tw_lo,
                                                      const float2 *__restrict__ tw_hi, int log2n,
                                                      int log2cols, long long tiles, long long total, float sgn) {
    constexpr int len = 1 << LOG2LEN;
    constexpr int LTC = clog2(TC);
    extern __shared__ float4 lds_raw[];
    float2 *buf = reinterpret_cast<float2 *>(lds_raw);
    const long long cols = 1LL << log2cols;
    // pass A: the twiddle tables after the tile; both passes: then the stage
    // twiddle bases
    float2 *tlo = buf + tile_vals(LOG2LEN, TC), *thi = tlo + 1024, *tht = thi + 1024;
    float2 *twl = PASS_A ? tht + 8 : tlo;
    static_assert(fft_tw_entries<R, LOG2LEN>() == tile_stage_tw_vals(R, LOG2LEN), "stage base count");
    if constexpr (PASS_A) tile_tables_to_lds(tlo, thi, tht, tw_lo, tw_hi);
    fft_tw_to_lds<R, LOG2LEN>(twl, tw);
    // this workgroup's tiles: t = first, first + step, ... < end (first < end:
    // the grid never exceeds the tiles)
    const long long G = gridDim.x, b = blockIdx.x;
    long long t = b;
    const long long step = G, end = total;
    if (G % (8 * (TC < 16 ? 16 / TC : 1)) == 0 && total % G == 0) t = tile_order<TC>(b);
    const TileWalk<TC> walk(G, tiles);
    long long tile = WALK ? walk.first(t) : t;  // the tile at walk position t
    int h = 0;
    float2 pre[R];
    tile_load_rows<R, LOG2LEN, TC>(pre, tile_rsrc(in, tile, end, tiles, TC, log2n), (int)cols, (int)threadIdx.x);
    auto one_tile = [&](long long cur) {
        // an empty asm that claims to change tx keeps the compiler from
        // hoisting every tx-derived address out of the tile loop and keeping
        // it live (which spills)
        int tx = (int)threadIdx.x;
        asm volatile("" : "+v"(tx));
        __syncthreads();  // the previous tile's LDS reads (or the tables' writes) are done
        const int c = tx & (TC - 1), e0 = tx >> LTC;
#pragma unroll
        for (int k = 0; k < R; ++k) buf[TileLayout<R, LOG2LEN, TC>::slot_k(c, e0, k * (len / R))] = pre[k];
        long long cur_tile = cur, next_tile = cur + step;
        if constexpr (WALK) {
            cur_tile = tile;
            tile = walk.next(tile, h);  // the walk's next step
            h = walk.next_h(h);
            next_tile = cur + step < end ? tile : end;
        }
        const TilePrefetch<R, LOG2LEN, TC> nxt{pre, tile_rsrc(in, next_tile, end, tiles, TC, log2n), (int)cols, tx};
        tile_load_rows<R, LOG2LEN, TC, 0, TilePrefetch<R, LOG2LEN, TC>::NC>(pre, nxt.r, nxt.cols, tx);
        const long long prob = cur_tile / tiles;
        const int c0 = (int)(cur_tile % tiles) * TC;
        tile_transform_store<R, LOG2LEN, PASS_A, TC, true>(buf, tlo, thi, tht, out, prob << log2n, c0, cols, log2n,
                                                           sgn, twl, tx, nxt);
    };
    one_tile(t);
    for (t += step; t < end; t += step) one_tile(t);
}

using TileKernel = void (*)(const float2 *, float2 *, const float2 *, const float2 *, const float2 *, int, int,
                            long long, long long, float);

constexpr int kTileLdsMax = 160 * 1024;
// LDS bytes of a pass: the tile, plus the twiddle tables in pass A, plus the
// stage twiddle bases in the persistent pass A
constexpr int64_t tile_lds(int radix, int log2len, int tc, bool pass_a) {
    return ((int64_t)tile_vals(log2len, tc) + (pass_a ? kTwLargeVals : 0) +
            (tile_persistent(log2len, tc, pass_a) ? tile_stage_tw_vals(radix, log2len) : 0)) *
           (int64_t)sizeof(float2);
}
// Tile shapes: radix 8 or 16; 64 to 1024 threads; the LDS budget (pass A
// with its tables).
constexpr bool tile_ok(int radix, int log2len, int tc, bool pass_a) {
    return (radix == 8 || radix == 16) && log2len >= clog2(radix) && tc * ((1 << log2len) / radix) >= 64 &&
           tc * ((1 << log2len) / radix) <= 1024 && tile_lds(radix, log2len, tc, pass_a) <= kTileLdsMax;
}

// walk: the persistent kernel with the whole-row step order (TileWalk), for
// launches where it reorders; shapes that are not persistent ignore it.
template <int R, int L, bool A, int TC>
static TileKernel tile_entry(bool walk) {
    if constexpr (!tile_ok(R, L, TC, A)) return nullptr;
    else if constexpr (tile_persistent(L, TC, A))
        return walk ? &k_fft_tile_p<R, L, A, TC, true> : &k_fft_tile_p<R, L, A, TC>;
    else return &k_fft_tile<R, L, A, TC>;
}
template <int R, bool A, int TC>
static TileKernel tile_len(int log2len, bool walk) {
    switch (log2len) {
        case 5: return tile_entry<R, 5, A, TC>(walk);
        case 6: return tile_entry<R, 6, A, TC>(walk);
        case 7: return tile_entry<R, 7, A, TC>(walk);
        case 8: return tile_entry<R, 8, A, TC>(walk);
        case 9: return tile_entry<R, 9, A, TC>(walk);
        case 10: return tile_entry<R, 10, A, TC>(walk);
        case 11: return tile_entry<R, 11, A, TC>(walk);
        case 12: return tile_entry<R, 12, A, TC>(walk);
        case 13: return tile_entry<R, 13, A, TC>(walk);
        default: return nullptr;
    }
}
template <int R, bool A>
static TileKernel tile_tc(int log2len, int tc, bool walk) {
    switch (tc) {
        case 2: return tile_len<R, A, 2>(log2len, walk);
        case 4: return tile_len<R, A, 4>(log2len, walk);
        case 8: return tile_len<R, A, 8>(log2len, walk);
        case 16: return tile_len<R, A, 16>(log2len, walk);
        case 32: return tile_len<R, A, 32>(log2len, walk);
        case 64: return tile_len<R, A, 64>(log2len, walk);
        default: return nullptr;
    }
}
template <bool A>
static TileKernel tile_lookup(int radix, int log2len, int tc, bool walk = false) {
    if (radix == 16) return tile_tc<16, A>(log2len, tc, walk);
    if (radix == 8) return tile_tc<8, A>(log2len, tc, walk);
    return nullptr;
}

const void *fft_tile_kernel(int radix, int log2len, int tc, bool pass_a) {
    return reinterpret_cast<const void *>(pass_a ? tile_lookup<true>(radix, log2len, tc)
                                                 : tile_lookup<false>(radix, log2len, tc));
}

bool fft_tile_shape_valid(int radix, int log2len, int tc, bool pass_a) {
    return (pass_a ? tile_lookup<true>(radix, log2len, tc) : tile_lookup<false>(radix, log2len, tc)) != nullptr;
}

int64_t fft_tile_lds_bytes(int radix, int log2len, int tc, bool pass_a) { return tile_lds(radix, log2len, tc, pass_a); }

void fft_large_host_twiddles(float *lo2, float *hi2) {
    const double two_pi = 6.283185307179586476925286766559;
    for (int j = 0; j < 1024; ++j) {
        const double a = two_pi * (double)j / (double)(1 << kLog2NLargeMax), b = two_pi * (double)j / 8192.0;
        lo2[2 * j] = (float)cos(a);
        lo2[2 * j + 1] = (float)(-sin(a));
        hi2[2 * j] = (float)cos(b);
        hi2[2 * j + 1] = (float)(-sin(b));
    }
    for (int j = 0; j < 8; ++j) {  // w_8^j
        const double c = two_pi * (double)j / 8.0;
        hi2[2 * (1024 + j)] = (float)cos(c);
        hi2[2 * (1024 + j) + 1] = (float)(-sin(c));
    }
}

// ---------------------------------------------------------------- plans

int fft_plan_check(int64_t n, const ppx_fft_plan &p) {
    if (!is_pow2(n) || n <= PPX_MAX_N || n > PPX_MAX_N_LARGE)
        return fail(PPX_EINVAL, "large FFT: n must be a power of two in (16384, 8388608]");
    const int ln = ilog2(n);
    if (p.log2_n1 < 1 || p.log2_n1 >= ln) return fail(PPX_ECONFIG, "plan: log2_n1 out of range");
    if (!fft_tile_shape_valid(p.radix_a, ln - p.log2_n1, p.tile_a, true))
        return fail(PPX_ECONFIG, "plan: no pass-A tile kernel for this radix / tile width and column length n / n1");
    if (!fft_tile_shape_valid(p.radix_b, p.log2_n1, p.tile_b, false))
        return fail(PPX_ECONFIG, "plan: no pass-B tile kernel for this radix / tile width and column length n1");
    if ((int64_t(1) << p.log2_n1) % p.tile_a || (n >> p.log2_n1) % p.tile_b)
        return fail(PPX_ECONFIG, "plan: tile width exceeds the number of columns");
    return PPX_OK;
}

std::vector<ppx_fft_plan> fft_enumerate_plans(int64_t n) {
    std::vector<ppx_fft_plan> out;
    if (!is_pow2(n) || n <= PPX_MAX_N || n > PPX_MAX_N_LARGE) return out;
    const int ln = ilog2(n);
    for (int l1 = 1; l1 < ln; ++l1)
        for (int ra : {8, 16})
            for (int rb : {8, 16})
                for (int ta : {2, 4, 8, 16, 32, 64})
                    for (int tb : {2, 4, 8, 16, 32, 64}) {
                        const ppx_fft_plan p{l1, ra, rb, ta, tb};
                        if (fft_tile_shape_valid(ra, ln - l1, ta, true) && fft_tile_shape_valid(rb, l1, tb, false) &&
                            (int64_t(1) << l1) % ta == 0 && (n >> l1) % tb == 0)
                            out.push_back(p);
                    }
    return out;
}

// The most even valid split (n1 <= n2 on a tie) and, in each pass, the
// widest tile of at most 16 columns, with radix 8 where both radices allow it.
void fft_default_plan(int64_t n, ppx_fft_plan &p) {
    const int ln = ilog2(n);
    p = ppx_fft_plan{0, 0, 0, 0, 0};
    auto pick = [&](int log2len, int64_t ncols, bool pass_a, int &radix, int &tile) {
        for (int t : {16, 8, 4, 2})
            for (int r : {8, 16})
                if (fft_tile_shape_valid(r, log2len, t, pass_a) && ncols % t == 0) {
                    radix = r;
                    tile = t;
                    return true;
                }
        return false;
    };
    int best = 1 << 30;
    for (int l1 = 1; l1 < ln; ++l1) {
        const int uneven = 2 * std::abs(2 * l1 - ln) + (2 * l1 > ln ? 1 : 0);
        int ra, ta, rb, tb;
        if (uneven < best && pick(ln - l1, int64_t(1) << l1, true, ra, ta) && pick(l1, n >> l1, false, rb, tb)) {
            p = ppx_fft_plan{l1, ra, rb, ta, tb};
            best = uneven;
        }
    }
}

namespace {
std::mutex g_plan_mu;
std::map<int64_t, ppx_fft_plan> g_plans;  // tuned plans by n
}  // namespace

bool fft_tuned_plan(int64_t n, ppx_fft_plan &p) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(n);
    if (it == g_plans.end()) return false;
    p = it->second;
    return true;
}

void fft_record_plan(int64_t n, const ppx_fft_plan &p) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans[n] = p;
}

std::vector<std::pair<int64_t, ppx_fft_plan>> fft_recorded_plans() {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    return std::vector<std::pair<int64_t, ppx_fft_plan>>(g_plans.begin(), g_plans.end());
}

void fft_clear_plans() {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans.clear();
}

int launch_fft_large(const void *in, void *out, int log2n, int64_t batch, const ppx_fft_plan &p, bool inverse,
                     hipStream_t s) {
    const DeviceInfo *di = device_info();
    if (!di) return PPX_EDEVICE;
    const int l1 = p.log2_n1, l2 = log2n - l1;
    const float sgn = inverse ? -1.0f : 1.0f;
    const float2 *tw = static_cast<const float2 *>(di->twiddles);
    const float2 *lo = static_cast<const float2 *>(di->twiddles_large_lo);
    const float2 *hi = static_cast<const float2 *>(di->twiddles_large_hi);
    // pass A: columns of length n2 of the [n2][n1] input, tiles of the n1 columns
    const long long tiles_a = (1LL << l1) / p.tile_a, tiles_b = (1LL << l2) / p.tile_b;
    const long long total_a = batch * tiles_a, total_b = batch * tiles_b;
    // persistent shapes: one workgroup per CU at most
    auto grid = [&](long long total, int log2len, int tc, bool pass_a) {
        return tile_persistent(log2len, tc, pass_a) ? std::min<long long>(total, std::max(di->cus, 1)) : total;
    };
    const bool walk_a = tile_walk_reorders(grid(total_a, l2, p.tile_a, true), tiles_a, p.tile_a);
    const bool walk_b = tile_walk_reorders(grid(total_b, l1, p.tile_b, false), tiles_b, p.tile_b);
    TileKernel ka = tile_lookup<true>(p.radix_a, l2, p.tile_a, walk_a);
    TileKernel kb = tile_lookup<false>(p.radix_b, l1, p.tile_b, walk_b);
    if (!ka || !kb) return fail(PPX_ECONFIG, "no tile kernel for this plan");
    hipLaunchKernelGGL(ka, dim3((unsigned)grid(total_a, l2, p.tile_a, true)), dim3(p.tile_a * ((1 << l2) / p.radix_a)),
                       (size_t)tile_lds(p.radix_a, l2, p.tile_a, true), s, static_cast<const float2 *>(in), static_cast<float2 *>(out),
                       tw, lo, hi, log2n, l1, tiles_a, total_a, sgn);
    int rc = fail_hip(hipGetLastError(), "large FFT pass A launch");
    if (rc) return rc;
    // pass B: columns of length n1 of the [n1][n2] intermediate, in place
    hipLaunchKernelGGL(kb, dim3((unsigned)grid(total_b, l1, p.tile_b, false)), dim3(p.tile_b * ((1 << l1) / p.radix_b)),
                       (size_t)tile_lds(p.radix_b, l1, p.tile_b, false), s, static_cast<const float2 *>(out), static_cast<float2 *>(out),
                       tw, lo, hi, log2n, l2, tiles_b, total_b, sgn);
    return fail_hip(hipGetLastError(), "large FFT pass B launch");
}

}  // namespace ppx
