// Batched complex FFT, Stockham autosort formulation (Sec. III of
// arXiv:2310.16214; radix r tunable, Sec. IV-A/V-C), for gfx950.
//
// A workgroup of L threads transforms G_b problems of size n; each problem is
// owned by T = n/P consecutive threads and thread `tid` of a problem always
// holds the P elements X[tid + j*T], j < P.  Stage s (radix RS, span Ns =
// product of the earlier radices) performs, for every butterfly t < n/RS with
// k = t mod Ns:
//     u_q = X[t + q*n/RS] * w_{Ns*RS}^{q*k},  u = DFT_RS(u),
//     Y[(t div Ns)*Ns*RS + k + q*Ns] = u_q,   q < RS,
// so each thread does P/RS butterflies per stage, and its inputs are exactly
// the P values it holds.  When log2 n is not a multiple of log2 r the first
// stage uses radix 2^(log2 n mod log2 r) (mixed radix).  The first stage reads
// global memory directly (consecutive threads read consecutive elements), the
// last writes global memory directly (likewise coalesced), and the stages in
// between exchange through LDS: either complex values, or -- to halve the LDS
// footprint (Sec. V-C) -- the real parts and then the imaginary parts through
// one float buffer.  Twiddles come from one table of w_NMAX^m held in global
// memory (cache resident), computed on the host in double precision.
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"
#include "ppx_internal.h"

namespace ppx {

constexpr int kNMax = 1 << kFftLog2NMax;

// LDS index swizzles that keep the strided Stockham writes free of bank
// conflicts without padding.  They act on the workgroup-flat index (problem
// offset included), so the problems sharing a workgroup land on different
// banks too; each keeps an index inside its aligned 256 (float2) or 1024
// (float) block, hence inside its problem for n >= that block and inside the
// workgroup's buffer always.
__device__ __forceinline__ int swz_c(int p) { return p ^ ((p >> 4) & 15); }  // float2 words
__device__ __forceinline__ int swz_f(int p) { return p ^ ((p >> 5) & 31); }  // float words

// The same swizzles with the block index shifted left by sigma before the
// XOR: p ^ (((p >> 4) << sigma) & 15) (float2), p ^ (((p >> 5) << sigma) & 31)
// (float).  A radix-RS stage with span 2^lns writes, per group of lanes served
// together (16 lanes of 8-byte words, 32 of 4-byte words), addresses whose
// low bits come partly from the lane index directly and partly from the
// block index (the lane bits at and above lns land log2 RS positions higher).
// sigma = min(lns, 4 - log2 RS) (float2) or min(lns, 5 - log2 RS) (float)
// moves those block-index bits onto exactly the low positions the lanes leave
// free, so every group's writes hit distinct banks; the reads of the same
// exchange (consecutive lanes on consecutive words) are conflict-free under
// any such swizzle.  sigma = 0 is the plain swizzle above (radix 16 with
// float2 words); radix 8 needs sigma = 1 after its first stage.
__device__ __forceinline__ int swz_cs(int p, int sigma) { return p ^ ((p >> (4 - sigma)) & ((15 << sigma) & 15)); }
__device__ __forceinline__ int swz_fs(int p, int sigma) { return p ^ ((p >> (5 - sigma)) & ((31 << sigma) & 31)); }

// Twiddles w[q] = w_{Ns*RS}^{q*k}, q = 1..RS-1, from the table of w_NMAX^m:
// w^k, w^{4k} and w^{8k} are read (as the radix needs them) and the other
// powers are products of at most three of them, so a butterfly issues at most
// three table loads instead of RS - 1.
// The table entries a radix-RS butterfly reads: w^k, w^{4k}, w^{8k}.
struct TwBase {
    float2 w1, w4, w8;
};
template <int RS>
__device__ __forceinline__ TwBase stage_twiddle_base(const float2 *__restrict__ tw, int k, int shift) {
    TwBase b;
    b.w1 = tw[k << shift];
    if constexpr (RS >= 8) b.w4 = tw[(4 * k) << shift];
    if constexpr (RS >= 16) b.w8 = tw[(8 * k) << shift];
    return b;
}
template <int RS>
__device__ __forceinline__ void stage_twiddles_from(float2 (&w)[RS], const TwBase &b) {
    w[1] = b.w1;
    if constexpr (RS >= 4) {
        w[2] = cmul(w[1], w[1]);
        w[3] = cmul(w[2], w[1]);
    }
    if constexpr (RS >= 8) {
        w[4] = b.w4;
        w[5] = cmul(w[4], w[1]);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
    }
    if constexpr (RS >= 16) {
        w[8] = b.w8;
#pragma unroll
        for (int q = 9; q < 16; ++q) w[q] = cmul(w[8], w[q - 8]);
    }
}
template <int RS>
__device__ __forceinline__ void stage_twiddles(float2 (&w)[RS], const float2 *__restrict__ tw, int k,
                                               int shift) {
    stage_twiddles_from<RS>(w, stage_twiddle_base<RS>(tw, k, shift));
}

// The first stage (span 1) has no twiddles; it is a separate instantiation
// (FIRST) rather than a runtime branch, so no control-flow join surrounds the
// twiddle products.  (gfx950 code generation with packed-FP32 selection off
// dropped the join copies of such a branch in the radix-4 kernel, feeding
// untwiddled imaginary parts to the butterfly.)
template <int RS, int P, bool FIRST>
__device__ __forceinline__ void stage_butterflies(float2 (&v)[P], int tid, int T, int lns,
                                                  const float2 *__restrict__ tw) {
    constexpr int NB = P / RS;
    constexpr int LRS = RS == 2 ? 1 : RS == 4 ? 2 : RS == 8 ? 3 : 4;
    const int twshift = kFftLog2NMax - (lns + LRS);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        float2 u[RS];
#pragma unroll
        for (int q = 0; q < RS; ++q) u[q] = v[i + q * NB];
        if constexpr (!FIRST) {
            const int k = (tid + i * T) & ((1 << lns) - 1);
            float2 w[RS];
            stage_twiddles<RS>(w, tw, k, twshift);
#pragma unroll
            for (int q = 1; q < RS; ++q) u[q] = cmul(u[q], w[q]);
        }
        RegDFT<RS>::run(u);
#pragma unroll
        for (int q = 0; q < RS; ++q) v[i + q * NB] = u[q];
    }
}

// Output position (within the problem) of slot (i, q) after a stage.
template <int RS>
__device__ __forceinline__ int stage_out_pos(int t, int lns, int q) {
    constexpr int LRS = RS == 2 ? 1 : RS == 4 ? 2 : RS == 8 ? 3 : 4;
    const int k = t & ((1 << lns) - 1);
    return ((t >> lns) << (lns + LRS)) + k + (q << lns);
}

// `lds` is the workgroup's buffer and `poff` the problem's offset in it.  The
// stage's swizzle (swz_cs / swz_fs with its sigma) is used for both the
// writes and the reads of the exchange.
template <int RS, int P, bool SPLIT>
__device__ __forceinline__ void stage_exchange(float2 (&v)[P], void *lds, int poff, int tid, int T,
                                               int lns) {
    constexpr int NB = P / RS;
    constexpr int LRS = RS == 2 ? 1 : RS == 4 ? 2 : RS == 8 ? 3 : 4;
    if constexpr (!SPLIT) {
        float2 *buf = static_cast<float2 *>(lds);
        const int sg = min(lns, 4 - LRS);
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int q = 0; q < RS; ++q)
                buf[swz_cs(poff + stage_out_pos<RS>(tid + i * T, lns, q), sg)] = v[i + q * NB];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = buf[swz_cs(poff + tid + j * T, sg)];
        __syncthreads();
    } else {
        float *buf = static_cast<float *>(lds);
        const int sg = min(lns, 5 - LRS);
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int q = 0; q < RS; ++q)
                buf[swz_fs(poff + stage_out_pos<RS>(tid + i * T, lns, q), sg)] = v[i + q * NB].x;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < P; ++j) v[j].x = buf[swz_fs(poff + tid + j * T, sg)];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int q = 0; q < RS; ++q)
                buf[swz_fs(poff + stage_out_pos<RS>(tid + i * T, lns, q), sg)] = v[i + q * NB].y;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < P; ++j) v[j].y = buf[swz_fs(poff + tid + j * T, sg)];
        __syncthreads();
    }
}

// The last stage's stores.  The T threads of a problem write T consecutive
// values per store instruction; where that run is at least kFftNtRun bytes
// the stores are non-temporal (kStoreNT), else default: with runs of 8 or 16
// bytes every instruction writes small pieces of many lines, and the
// streaming hint sends each piece to memory on its own (n = 16 at one thread
// per problem measured 3.6x slower with it).
constexpr int kFftNtRun = 32;
__device__ __forceinline__ bool fft_nt_stores(int T) { return T * (int)sizeof(float2) >= kFftNtRun; }

template <int RS, int P>
__device__ __forceinline__ void stage_store(const float2 (&v)[P], float2 *dst, int tid, int T,
                                            int lns, float sgn) {
    constexpr int NB = P / RS;
    if (fft_nt_stores(T)) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                const float2 o = v[i + q * NB];
                store_nt_any(dst + stage_out_pos<RS>(tid + i * T, lns, q), make_float2(o.x, sgn * o.y));
            }
    } else {
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                const float2 o = v[i + q * NB];
                dst[stage_out_pos<RS>(tid + i * T, lns, q)] = make_float2(o.x, sgn * o.y);
            }
    }
}

// One stage of radix RS followed by either the LDS exchange or, for the last
// stage, the global store.
template <int RS, int P, bool SPLIT, bool FIRST>
__device__ __forceinline__ void run_stage(float2 (&v)[P], void *lds, int poff, float2 *dst, int tid,
                                          int T, int &lns, int log2n, bool active, float sgn,
                                          const float2 *__restrict__ tw) {
    constexpr int LRS = RS == 2 ? 1 : RS == 4 ? 2 : RS == 8 ? 3 : 4;
    stage_butterflies<RS, P, FIRST>(v, tid, T, lns, tw);
    if (lns + LRS == log2n) {
        if (active) stage_store<RS, P>(v, dst, tid, T, lns, sgn);
    } else {
        stage_exchange<RS, P, SPLIT>(v, lds, poff, tid, T, lns);
    }
    lns += LRS;
}

// One workgroup's share: problems [p0, p0 + nprob) with the workgroup's
// threads laid out as problems of T = n/P threads (threads of problems beyond
// nprob only take part in the barriers).  `lds_raw` holds at least
// (blockDim.x * P / n) problems.  Used by k_fft and by the fused kernel.
template <int R, int P, bool SPLIT>
__device__ __forceinline__ void fft_block(const float2 *in, float2 *out, const float2 *__restrict__ tw,
                                          int log2n, long long p0, int nprob, float sgn,
                                          void *lds_raw) {
    constexpr int LR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
    const int n = 1 << log2n;
    const int lT = log2n - (P == 2 ? 1 : P == 4 ? 2 : P == 8 ? 3 : P == 16 ? 4 : 5);
    const int T = 1 << lT;
    const int lp = threadIdx.x >> lT;
    const int tid = threadIdx.x & (T - 1);
    const long long prob = p0 + lp;
    const bool active = lp < nprob;
    const float2 *src = in + prob * n;
    float2 *dst = out + prob * n;
    const int poff = lp * n;  // the problem's offset in the workgroup's LDS buffer

    float2 v[P];
    if (active) {
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = src[tid + j * T];
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = make_float2(0.f, 0.f);
    }
    // all P loads in flight before the first use (the conjugation of the
    // inverse transform would otherwise be interleaved with them)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < P; ++j) v[j].y *= sgn;

    // first stage: radix 2^(log2 n mod log2 R) when R does not divide log2 n
    int lns = 0;
    const int rem = log2n % LR;
    if (rem == 0) {
        run_stage<R, P, SPLIT, true>(v, lds_raw, poff, dst, tid, T, lns, log2n, active, sgn, tw);
    } else if (rem == 1) {
        run_stage<2, P, SPLIT, true>(v, lds_raw, poff, dst, tid, T, lns, log2n, active, sgn, tw);
    } else if constexpr (R >= 8) {
        if (rem == 2) run_stage<4, P, SPLIT, true>(v, lds_raw, poff, dst, tid, T, lns, log2n, active, sgn, tw);
        if constexpr (R >= 16)
            if (rem == 3) run_stage<8, P, SPLIT, true>(v, lds_raw, poff, dst, tid, T, lns, log2n, active, sgn, tw);
    }
    while (lns < log2n)
        run_stage<R, P, SPLIT, false>(v, lds_raw, poff, dst, tid, T, lns, log2n, active, sgn, tw);
}

template <int R, int P, bool SPLIT>
__global__ __launch_bounds__(fft_max_threads(P)) void k_fft(const float2 *in, float2 *out,
                                                             const float2 *__restrict__ tw, int log2n,
                                                             long long batch, int gb, float sgn) {
    extern __shared__ float4 lds_raw[];
    const long long p0 = (long long)blockIdx.x * gb;
    const int nprob = (int)min((long long)gb, batch - p0);
    fft_block<R, P, SPLIT>(in, out, tw, log2n, p0, nprob, sgn, lds_raw);
}

// ---------------------------------------------------------------------------
// Kernels specialised on log2 n (radix R = P, the shape the tuners pick for
// n >= 128): with n a constant, the stage sequence is unrolled at compile
// time, every index offset (j*T, q << lns) is a constant, and where a
// constant has no bits in 4..7 the swizzle commutes with it, so most LDS and
// global addresses become one base register plus an immediate.  This removes
// most of the integer work and about a third of the registers of the generic
// kernel; the transform is the same.
constexpr int clog2(int x) { return x <= 1 ? 0 : 1 + clog2(x / 2); }

// With STAGED the last stage leaves its results in the LDS buffer, at their
// output positions (XORed with pxor, then swizzled), instead of storing them
// (see k_fft_n).  A nonzero pxor needs pxor < 64 <= T and a last stage whose
// span is at least 64: the XOR is then applied to the thread index, where it
// changes the same low bits of the position.  With a last span of at least 64
// and one butterfly per thread, poff must be a multiple of 256.  After the
// exchange that follows stage s (0-based), hook.template at<s>() runs: a
// caller's work to place between the stages (none by default).
struct NoStageHook {
    template <int S>
    __device__ __forceinline__ void at() const {}
};
template <int R, int P, bool SPLIT, int LOG2N, int LNS, bool STAGED = false, typename Hook = NoStageHook>
__device__ __forceinline__ void fft_stages_ct(float2 (&v)[P], void *lds, int poff, float2 *dst, int tid,
                                              bool active, float sgn, const float2 *__restrict__ tw,
                                              const Hook &hook = Hook{}, int pxor = 0) {
    constexpr int REM = LOG2N % clog2(R);
    constexpr int RS = (LNS == 0 && REM != 0) ? (1 << REM) : R;  // mixed-radix first stage
    constexpr int LRS = clog2(RS);
    constexpr int T = 1 << (LOG2N - clog2(P));
    stage_butterflies<RS, P, LNS == 0>(v, tid, T, LNS, tw);
    if constexpr (LNS + LRS == LOG2N) {
        if constexpr (STAGED) {
            constexpr int NB = P / RS;
            float2 *buf = static_cast<float2 *>(lds);
            if constexpr (NB == 1 && LNS >= 6) {
                // position t + q 2^LNS (t = tid ^ pxor < 2^LNS); with poff a
                // multiple of 256, its swizzle is that of poff + t XORed with
                // the swizzle term of q 2^LNS (bits 4..7 moved to 0..3), plus
                // q 2^LNS: one base, constant offsets
                const int b = swz_c(poff + (tid ^ pxor));
#pragma unroll
                for (int q = 0; q < RS; ++q) buf[(b ^ (((q << LNS) >> 4) & 15)) + (q << LNS)] = v[q];
            } else {
#pragma unroll
                for (int i = 0; i < NB; ++i)
#pragma unroll
                    for (int q = 0; q < RS; ++q)
                        buf[swz_c(poff + stage_out_pos<RS>((tid ^ pxor) + i * T, LNS, q))] = v[i + q * NB];
            }
        } else {
            if (active) stage_store<RS, P>(v, dst, tid, T, LNS, sgn);
        }
    } else {
        stage_exchange<RS, P, SPLIT>(v, lds, poff, tid, T, LNS);
        // index of the stage just done: the first spans REM or log2 R bits
        constexpr int S = LNS == 0 ? 0 : 1 + (LNS - (REM ? REM : clog2(R))) / clog2(R);
        hook.template at<S>();
        fft_stages_ct<R, P, SPLIT, LOG2N, LNS + LRS, STAGED, Hook>(v, lds, poff, dst, tid, active, sgn, tw, hook,
                                                                   pxor);
    }
}

// Global I/O staged through LDS, for small n: the workgroup's G_b * n
// contiguous values are read (and at the end written) as one sweep of
// 16-byte words, consecutive lanes on consecutive words, and rearranged in
// the exchange buffer.  Direct accesses would move runs of only T values per
// problem per instruction (T = n / P <= 16 here).  Used where the exchange
// buffer holds complex values (not SPLIT), there is an exchange (n > radix)
// and n <= 64.  Inside whole benchmark steps this took n = 16 from 117 to 92
// us and n = 32 from 105 to 92 us per 256 MiB call; from n = 256 on the two
// extra LDS passes cost more than they save.
template <int R, int P, bool SPLIT, int LOG2N>
constexpr bool fft_staged_io() {
    return !SPLIT && LOG2N <= 6 && LOG2N > clog2(R) && (1 << (LOG2N - clog2(P))) <= 16;
}

// Words [0, total/2) of the block into the buffer (swizzled float2 slots);
// tx is the thread's index in the workgroup, nt the workgroup's threads.
__device__ __forceinline__ void fft_stage_in(float2 *buf, const float2 *src, int total, int tx, int nt) {
    const float4 *src4 = reinterpret_cast<const float4 *>(src);
    for (int e = tx; 2 * e < total; e += nt) {
        const float4 w = src4[e];
        buf[swz_c(2 * e)] = make_float2(w.x, w.y);
        buf[swz_c(2 * e + 1)] = make_float2(w.z, w.w);
    }
}

// The buffer's first total values to dst as 16-byte words (conjugated for the
// inverse transform), with non-temporal stores.
__device__ __forceinline__ void fft_stage_out(const float2 *buf, float2 *dst, int total, float sgn, int tx,
                                              int nt) {
    u32x4 *dst4 = reinterpret_cast<u32x4 *>(dst);
    for (int e = tx; 2 * e < total; e += nt) {
        const float2 a = buf[swz_c(2 * e)], b = buf[swz_c(2 * e + 1)];
        store_nt(dst4 + e, __builtin_bit_cast(u32x4, make_float4(a.x, sgn * a.y, b.x, sgn * b.y)));
    }
}

// The thread's slots X[tid + j*T] as stored (zeros for threads beyond the
// group's problems).  All P loads are issued before anything consumes them.
template <int P, int LOG2N>
__device__ __forceinline__ void fft_load_raw_ct(float2 (&v)[P], const float2 *src, int tid, bool active) {
    constexpr int T = 1 << (LOG2N - clog2(P));
    if (active) {
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = src[tid + j * T];
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = make_float2(0.f, 0.f);
    }
}

// Conjugation of the inputs for the inverse transform (sgn = -1).
template <int P>
__device__ __forceinline__ void fft_conj(float2 (&v)[P], float sgn) {
#pragma unroll
    for (int j = 0; j < P; ++j) v[j].y *= sgn;
}

// One workgroup's share with the log2 n-specialised stage sequence:
// problems [p0, p0 + nprob), laid out as in fft_block (T = n/P threads per
// problem; threads of problems beyond nprob only take part in the barriers).
// Used by k_fft_n and by the mixed launch's FFT tiles, so both compute the
// same values.  tx is the thread's index in the workgroup and nt the
// workgroup's threads (passed in, so that a caller's loop can keep the
// addresses derived from them from being hoisted and held in registers).
template <int R, int P, bool SPLIT, int LOG2N>
__device__ __forceinline__ void fft_group_ct(const float2 *in, float2 *out, const float2 *__restrict__ tw,
                                             long long p0, int nprob, float sgn, void *lds_raw, int tx, int nt) {
    constexpr int n = 1 << LOG2N;
    constexpr int lT = LOG2N - clog2(P);
    const int lp = tx >> lT;
    const int tid = tx & ((1 << lT) - 1);
    const long long prob = p0 + lp;
    const bool active = lp < nprob;
    float2 v[P];
    if constexpr (fft_staged_io<R, P, SPLIT, LOG2N>()) {
        // threads of problems beyond nprob transform stale buffer contents and
        // store nothing: the sweeps cover the nprob problems only
        constexpr int T = 1 << lT;
        float2 *buf = reinterpret_cast<float2 *>(lds_raw);
        const int total = nprob * n;
        fft_stage_in(buf, in + p0 * n, total, tx, nt);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = buf[swz_c(lp * n + tid + j * T)];
        __syncthreads();
        fft_conj<P>(v, sgn);
        fft_stages_ct<R, P, SPLIT, LOG2N, 0, true>(v, lds_raw, lp * n, nullptr, tid, active, sgn, tw);
        __syncthreads();
        fft_stage_out(buf, out + p0 * n, total, sgn, tx, nt);
    } else {
        fft_load_raw_ct<P, LOG2N>(v, in + prob * n, tid, active);
        // keep the scheduler from interleaving the loads with their first use,
        // which would leave only a few of them in flight
        __builtin_amdgcn_sched_barrier(0);
        fft_conj<P>(v, sgn);
        fft_stages_ct<R, P, SPLIT, LOG2N, 0>(v, lds_raw, lp * n, out + prob * n, tid, active, sgn, tw);
    }
}

// Same arguments as k_fft (log2n is implied by LOG2N).
template <int R, int P, bool SPLIT, int LOG2N>
__global__ __launch_bounds__(fft_max_threads(P)) void k_fft_n(const float2 *in, float2 *out,
                                                               const float2 *__restrict__ tw, int,
                                                               long long batch, int gb, float sgn) {
    extern __shared__ float4 lds_raw[];
    const long long p0 = (long long)blockIdx.x * gb;
    const int nprob = (int)min((long long)gb, batch - p0);
    fft_group_ct<R, P, SPLIT, LOG2N>(in, out, tw, p0, nprob, sgn, lds_raw, threadIdx.x, blockDim.x);
}

// --- persistent variant
//
// The twiddle-table entries every stage reads depend on the thread only, so
// the persistent kernel copies them into LDS (after the exchange buffer) once
// per workgroup and reads its bases from there.  Global twiddle reads inside
// the loop would be issued after the previous group's stores, and vector
// memory operations complete in issue order, so the first stage that needs a
// twiddle would wait for those stores; LDS reads use a separate counter.

template <int R, int LOG2N>
constexpr int fft_twiddled_stages() {
    return (LOG2N + clog2(R) - 1) / clog2(R) - 1;  // every stage but the first
}
// log2 of the span of twiddled stage i (the stage's lns)
template <int R, int LOG2N>
constexpr int fft_tw_lns(int i) {
    return (LOG2N % clog2(R) ? LOG2N % clog2(R) : clog2(R)) + i * clog2(R);
}
// table entries a radix-R butterfly reads per k: w^k, w^{4k}, w^{8k}
template <int R>
constexpr int fft_tw_per_k() { return 1 + (R >= 8) + (R >= 16); }
// LDS offset (float2 entries) of twiddled stage i's bases, and their total
template <int R, int LOG2N>
constexpr int fft_tw_offset(int i) {
    int off = 0;
    for (int j = 0; j < i; ++j) off += fft_tw_per_k<R>() << fft_tw_lns<R, LOG2N>(j);
    return off;
}
template <int R, int LOG2N>
constexpr int fft_tw_entries() { return fft_tw_offset<R, LOG2N>(fft_twiddled_stages<R, LOG2N>()); }

// Copies every stage's bases into twl: stage i, power p (1, 4, 8), k < span.
template <int R, int LOG2N>
__device__ __forceinline__ void fft_tw_to_lds(float2 *twl, const float2 *__restrict__ tw) {
    constexpr int NS = fft_twiddled_stages<R, LOG2N>();
    for (int e = threadIdx.x; e < fft_tw_entries<R, LOG2N>(); e += blockDim.x) {
        int i = 0;
#pragma unroll
        for (int j = 1; j < NS; ++j)
            if (e >= fft_tw_offset<R, LOG2N>(j)) i = j;
        int lns = 0, off = 0;
#pragma unroll
        for (int j = 0; j < NS; ++j)
            if (j == i) {
                lns = fft_tw_lns<R, LOG2N>(j);
                off = fft_tw_offset<R, LOG2N>(j);
            }
        const int r = e - off;
        const int pw = r >> lns;  // 0, 1, 2 -> w^k, w^{4k}, w^{8k}
        const int k = r & ((1 << lns) - 1);
        const int mult = pw == 0 ? 1 : pw == 1 ? 4 : 8;
        twl[e] = tw[(mult * k) << (kFftLog2NMax - (lns + clog2(R)))];
    }
}

// Chunk C of NC of the thread's loads X[tid + j*T] for a group: the loads j
// with j * NC / P == C (so the chunks partition the P loads).
template <int P, int LOG2N, int C, int NC>
__device__ __forceinline__ void fft_load_chunk(float2 (&v)[P], __amdgpu_buffer_rsrc_t r, int poff, int tid) {
    constexpr int T = 1 << (LOG2N - clog2(P));
    const int voff = (poff + tid) * (int)sizeof(float2);
#pragma unroll
    for (int j = 0; j < P; ++j)  // the constant part of the offset in the scalar operand
        if (j * NC / P == C)
            v[j] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(
                                                   r, voff, j * T * (int)sizeof(float2), 0));
}

template <int RS, int P, int POLICY>
__device__ __forceinline__ void stage_store_buf(const float2 (&v)[P], __amdgpu_buffer_rsrc_t r, int poff,
                                                int tid, int T, int lns, float sgn) {
    constexpr int NB = P / RS;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        // stage_out_pos(t, lns, q) = stage_out_pos(t, lns, 0) + (q << lns): the
        // q part goes in the scalar offset operand
        const int voff = (poff + stage_out_pos<RS>(tid + i * T, lns, 0)) * (int)sizeof(float2);
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            const float2 o = v[i + q * NB];
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, make_float2(o.x, sgn * o.y)), r, voff,
                                                  (q << lns) * (int)sizeof(float2), POLICY);
        }
    }
}

// The stages of one group, with the next group's loads (into nxt, from src)
// spread over them: stage s < NC issues chunk s of NC = (stages - 1) chunks,
// so none is issued in the last stage, just before the stores.
template <int R, int P, bool SPLIT, int LOG2N, int LNS, int IDX>
__device__ __forceinline__ void fft_stages_pre(float2 (&v)[P], const float2 *twl, void *lds, int poff,
                                               __amdgpu_buffer_rsrc_t dst, int tid, float sgn,
                                               float2 (&nxt)[P], __amdgpu_buffer_rsrc_t src) {
    constexpr int NST = (LOG2N + clog2(R) - 1) / clog2(R);
    constexpr int NC = NST > 1 ? NST - 1 : 1;
    constexpr int STAGE = LNS == 0 ? 0 : IDX + 1;
    if constexpr (STAGE < NC) {
        // the scheduler would otherwise gather every chunk at the loop top
        __builtin_amdgcn_sched_barrier(0);
        fft_load_chunk<P, LOG2N, STAGE, NC>(nxt, src, poff, tid);
        __builtin_amdgcn_sched_barrier(0);
    }
    constexpr int REM = LOG2N % clog2(R);
    constexpr int RS = (LNS == 0 && REM != 0) ? (1 << REM) : R;
    constexpr int LRS = clog2(RS);
    constexpr int T = 1 << (LOG2N - clog2(P));
    if constexpr (LNS == 0) {
        stage_butterflies<RS, P, true>(v, tid, T, 0, nullptr);
    } else {  // radix R = P: one butterfly per thread; bases from LDS
        constexpr int OFF = fft_tw_offset<R, LOG2N>(IDX);
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
    constexpr int NEXT_IDX = LNS == 0 ? IDX : IDX + 1;
    if constexpr (LNS + LRS == LOG2N) {
        stage_store_buf<RS, P, (T * (int)sizeof(float2) >= kFftNtRun ? kStoreNT : 0)>(v, dst, poff, tid, T, LNS, sgn);
    } else {
        stage_exchange<RS, P, SPLIT>(v, lds, poff, tid, T, LNS);
        fft_stages_pre<R, P, SPLIT, LOG2N, LNS + LRS, NEXT_IDX>(v, twl, lds, poff, dst, tid, sgn, nxt, src);
    }
}

// Persistent variant of k_fft_n: a grid of resident workgroups (at most one
// per group) walks the groups of gb problems (g, g + gridDim.x, ...) and loads
// the next group's inputs into a second register set while it transforms the
// current one, so a workgroup's global traffic overlaps its own stages.  This
// matters where the LDS buffer allows only one or two workgroups per CU
// (large n): otherwise a CU alternates between loading and computing.  The
// next group's loads are issued in chunks over the stages rather than all at
// once: measured at n = 16384 this takes 11% off the call (a burst of every
// load at the loop top, on the heels of the previous group's stores, left
// the memory system idle during the rest of the stages).
//
// Vector-memory operations complete in issue order, so the wait for the
// prefetched values must not also cover the stores issued after them; the
// code keeps the compiler's wait at exactly that point:
//  * loads and stores go through buffer descriptors, so no lane needs a
//    branch (a branch around a store or load makes the paths that meet after
//    it differ, and the wait after the join must cover the worse one);
//  * the first iteration is peeled, so the loop is entered only from paths
//    with the same history (prefetch, then stores) as its back edge, and the
//    loop body is unrolled twice with the two register sets swapping roles,
//    so no register copy (which would wait for the prefetch) is needed;
//  * the twiddle bases are read from LDS, not global memory;
//  * an empty asm that claims to change tid keeps the compiler from hoisting
//    every tid-derived address out of the loop and keeping it live, which
//    with the second register set spilled at 1024 threads.
// Every thread runs the same number of iterations, so all reach every barrier.
template <int R, int P, bool SPLIT, int LOG2N>
__global__ __launch_bounds__(fft_max_threads(P)) void k_fft_np(const float2 *in, float2 *out,
                                                                const float2 *__restrict__ tw, int,
                                                                long long batch, int gb, float sgn) {
    static_assert(R == P, "one butterfly per thread and stage");
    extern __shared__ float4 lds_raw[];
    constexpr int n = 1 << LOG2N;
    constexpr int lT = LOG2N - clog2(P);
    const int lp = threadIdx.x >> lT;
    const int tid0 = threadIdx.x & ((1 << lT) - 1);
    const int poff = lp * n;
    const long long ngroups = (batch + gb - 1) / gb;
    // the twiddle bases follow the exchange buffer (gb * n complex values, or
    // gb * n floats with the split exchange)
    float2 *twl = reinterpret_cast<float2 *>(reinterpret_cast<char *>(lds_raw) +
                                             (size_t)gb * n * (SPLIT ? sizeof(float) : sizeof(float2)));
    fft_tw_to_lds<R, LOG2N>(twl, tw);
    __syncthreads();

    long long g = blockIdx.x;  // < ngroups: the grid never exceeds the groups
    const long long G = gridDim.x;
    // Two register sets take turns (no copies between them): one iteration
    // transforms `cur` while the next group's loads land in `nxt`.
    float2 A[P], B[P];
    auto iteration = [&](long long grp, float2 (&cur)[P], float2 (&nxt)[P]) {
        int tid = tid0;
        asm volatile("" : "+v"(tid));
        fft_conj<P>(cur, sgn);
        fft_stages_pre<R, P, SPLIT, LOG2N, 0, 0>(cur, twl, lds_raw, poff,
                                                 group_rsrc(out, grp, gb, n, sizeof(float2), batch), tid, sgn,
                                                 nxt, group_rsrc(in, grp + G, gb, n, sizeof(float2), batch));
    };
    fft_load_chunk<P, LOG2N, 0, 1>(A, group_rsrc(in, g, gb, n, sizeof(float2), batch), poff, tid0);
    iteration(g, A, B);
    for (g += G; g < ngroups; g += 2 * G) {
        iteration(g, B, A);
        if (g + G >= ngroups) break;
        iteration(g + G, A, B);
    }
}

}  // namespace ppx
