// Batched inclusive and exclusive sum scans (Sec. III "Scan Operator" of
// arXiv:2310.16214), int32 (modulo 2^32), float32 and float64, for gfx950.
//
// A workgroup of L threads scans G_b problems of size n; problem p is owned by
// T = n/P consecutive threads and thread `tid` holds the P contiguous elements
// [tid*P, tid*P + P), so the workgroup's loads and stores are one contiguous,
// vectorised sweep over its G_b*n elements.  Steps:
//   1. thread-serial inclusive scan of the P values (registers);
//   2. inclusive scan of the thread totals across the lanes of each problem
//      segment (min(T, 64) lanes) with a wave64 lane network: Kogge-Stone
//      (DPP row shifts + row broadcasts) or Ladner-Fischer (swizzle
//      broadcasts) -- the two prefix circuits the paper tunes;
//   3. when a problem spans several waves (T > 64), each wave's total goes to
//      one LDS slot and every thread adds the totals of the earlier waves of
//      its problem (the paper's per-problem shared-memory slots, one per wave);
//   4. add the exclusive prefix to the P values and store; the thread's
//      prefix is the inclusive lane result of the lane before it, so every
//      term of an output is a sum of elements at or before that output.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"
#include "ppx_internal.h"

namespace ppx {

// P contiguous values as 16-byte words (8-byte ones where P values are
// fewer than 16 bytes' worth).
template <typename T, int P>
__device__ __forceinline__ void load_chunk(const T *src, T (&v)[P]) {
    constexpr int B = P * (int)sizeof(T);
    if constexpr (B % 16 == 0) {
        const int4 *s4 = reinterpret_cast<const int4 *>(src);
#pragma unroll
        for (int j = 0; j < B / 16; ++j) {
            const int4 w = s4[j];
            __builtin_memcpy(&v[j * 16 / (int)sizeof(T)], &w, 16);
        }
    } else {
        static_assert(B == 8, "8 bytes or a multiple of 16");
        const int2 w = *reinterpret_cast<const int2 *>(src);
        __builtin_memcpy(&v[0], &w, 8);
    }
}

template <typename T, int P>
__device__ __forceinline__ void store_chunk(T *dst, const T (&v)[P]) {
    constexpr int B = P * (int)sizeof(T);
    if constexpr (B % 16 == 0) {
        int4 *d4 = reinterpret_cast<int4 *>(dst);
#pragma unroll
        for (int j = 0; j < B / 16; ++j) {
            int4 w;
            __builtin_memcpy(&w, &v[j * 16 / (int)sizeof(T)], 16);
            d4[j] = w;
        }
    } else {
        static_assert(B == 8, "8 bytes or a multiple of 16");
        int2 w;
        __builtin_memcpy(&w, &v[0], 8);
        *reinterpret_cast<int2 *>(dst) = w;
    }
}

// Steps 1-4 on the P values a thread holds (lT = log2 threads per problem).
// `wave_tot` holds blockDim.x / 64 values; with T > 64 threads per problem
// there is one barrier, which every thread of the workgroup must reach.
// EXCL: the exclusive scan (each output the sum of the inputs before it):
// step 1 is then the thread-serial exclusive scan, the rest is unchanged.
// tx: the thread's index in the workgroup.
template <typename T, int P, int ALGO, bool EXCL = false, typename U>
__device__ __forceinline__ void scan_values(U (&v)[P], int lT, T *wave_tot, int tx) {
    // 1. serial scan within the thread
    U total;
    if constexpr (EXCL) {
        U run = U(0);
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const U x = v[j];
            v[j] = run;
            run = run + x;
        }
        total = run;
    } else {
#pragma unroll
        for (int j = 1; j < P; ++j) v[j] = v[j] + v[j - 1];
        total = v[P - 1];
    }

    // 2. lane network over the problem's segment of the wave
    const int lane = tx & (kWave - 1);
    const int seg = lT >= 6 ? kWave : (1 << lT);
    const U incl = ALGO == PPX_SCAN_LF ? lanes_scan_lf<U>(total, seg, lane)
                                       : lanes_scan_ks<U>(total, seg, lane);
    // Exclusive prefix of this thread within the segment: the previous lane's
    // inclusive value (0 at the segment's first lane), moved by a one-lane
    // shift.  Forming it as incl - total instead would cancel: every output
    // would then carry rounding on the scale of the thread's whole chunk and
    // of the elements after it, not of the sum the output is defined by.
    const U prev = dpp_wave_shr1(incl);
    U prefix = (lane & (seg - 1)) == 0 ? U(0) : prev;

    // 3. earlier waves of the same problem
    if (lT > 6) {
        const int w = tx >> 6;
        if (lane == kWave - 1) wave_tot[w] = __builtin_bit_cast(T, incl);
        __syncthreads();
        const int w0 = w & ~((1 << (lT - 6)) - 1);
        for (int u = w0; u < w; ++u) prefix = prefix + __builtin_bit_cast(U, wave_tot[u]);
    }

    // 4. add the prefix
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = v[j] + prefix;
}

// Integer adds wrap modulo 2^32: they are done on unsigned values.
template <typename T>
using ScanArith = typename std::conditional<std::is_same<T, int>::value, unsigned, T>::type;

// One workgroup's share: problems [p0, p0 + nprob), T = n/P threads per
// problem (threads of problems beyond nprob compute on zeros and store
// nothing).  `wave_tot` holds blockDim.x / 64 values; tx is the thread's
// index in the workgroup.  Used by k_scan and by the mixed launch's tiles.
template <typename T, int P, int ALGO, bool EXCL = false>
__device__ __forceinline__ void scan_block(const T *in, T *out, int log2n, long long p0, int nprob,
                                           T *wave_tot, int tx) {
    constexpr int LP = P == 2 ? 1 : P == 4 ? 2 : P == 8 ? 3 : P == 16 ? 4 : 5;
    using U = ScanArith<T>;
    const int lT = log2n - LP;  // log2 threads per problem
    const int lp = tx >> lT;
    const bool active = lp < nprob;
    const long long off = p0 * (1LL << log2n) + (long long)tx * P;

    U v[P];
    if (active) {
        load_chunk<U, P>(reinterpret_cast<const U *>(in) + off, v);
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = U(0);
    }
    scan_values<T, P, ALGO, EXCL>(v, lT, wave_tot, tx);
    if (active) store_chunk<U, P>(reinterpret_cast<U *>(out) + off, v);
}

template <typename T, int P, int ALGO, bool EXCL>
__global__ __launch_bounds__(1024) void k_scan(const T *in, T *out, int log2n, long long batch,
                                               int gb) {
    __shared__ T wave_tot[kMaxThreadsPerBlock / kWave];
    const long long p0 = (long long)blockIdx.x * gb;
    scan_block<T, P, ALGO, EXCL>(in, out, log2n, p0, (int)min((long long)gb, batch - p0), wave_tot, threadIdx.x);
}

// Persistent variant: a grid of resident workgroups (at most one per group)
// walks the groups of gb problems (g, g + gridDim.x, ...) and loads the next
// group's values into a second register set while it scans the current one,
// so the loads overlap the barrier-bound steps of workgroups that span many
// waves.  Loads and stores go through per-group buffer descriptors (lanes
// past the batch read zeros and store nothing, without a branch); the first
// iteration is peeled and the loop unrolled twice with the two register sets
// swapping roles, so the wait for the prefetched group never also covers the
// stores issued after it.  The wave totals alternate between two buffers: a
// wave may start the next group before a slower one has read this group's
// totals, and the barrier of every group keeps the waves within one group of
// each other.
template <typename T, int P, int ALGO, bool EXCL>
__global__ __launch_bounds__(1024) void k_scan_pipe(const T *in, T *out, int log2n, long long batch,
                                                    int gb) {
    constexpr int LP = P == 2 ? 1 : P == 4 ? 2 : P == 8 ? 3 : P == 16 ? 4 : 5;
    using U = ScanArith<T>;
    __shared__ T wave_tot[2][kMaxThreadsPerBlock / kWave];
    const int lT = log2n - LP;
    const long long n = 1LL << log2n;
    const int voff = threadIdx.x * P * (int)sizeof(T);  // byte offset within a group
    const long long ngroups = (batch + gb - 1) / gb;
    const long long G = gridDim.x;
    U v0[P], v1[P];
    auto iteration = [&](long long grp, int parity, U (&cur)[P], U (&nxt)[P]) {
        buf_load<U, P>(nxt, group_rsrc(in, grp + G, gb, n, sizeof(T), batch), voff);
        __builtin_amdgcn_sched_barrier(0);
        scan_values<T, P, ALGO, EXCL>(cur, lT, wave_tot[parity], threadIdx.x);
        buf_store<U, P>(cur, group_rsrc(out, grp, gb, n, sizeof(T), batch), voff);
    };
    long long g = blockIdx.x;  // < ngroups: the grid never exceeds the groups
    buf_load<U, P>(v0, group_rsrc(in, g, gb, n, sizeof(T), batch), voff);
    iteration(g, 0, v0, v1);
    for (g += G; g < ngroups; g += 2 * G) {
        iteration(g, 1, v1, v0);
        if (g + G >= ngroups) break;
        iteration(g + G, 0, v0, v1);
    }
}

}  // namespace ppx
