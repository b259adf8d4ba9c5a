// Launch-parameter space of the batched kernels: validity predicate,
// derived fields, enumeration, the plain "default" configuration and the
// tuned-configuration cache.
//
// The space is the paper's (Sec. IV-A, Sec. V and Table "parameters-TL"):
// radix r, elements per thread P, threads per block L and -- made explicit
// here -- problems per block G_b, tied by P * L = G_b * N.  The paper's
// "shuffle" switch has no separate field: on gfx950 the lane networks of the
// scan always run in registers, and the LDS use of each kernel follows from
// (N, G_b, algo).
#include <cstring>

#include "ppx_internal.h"

namespace ppx {

static bool is_valid_dtype(int op, int dtype) {
    switch (op) {
        case PPX_OP_FFT: return dtype == PPX_C64;
        case PPX_OP_SCAN: return dtype == PPX_I32 || dtype == PPX_F32 || dtype == PPX_F64;
        case PPX_OP_TRIDIAG: return dtype == PPX_F32 || dtype == PPX_F64;
        default: return false;
    }
}

static int64_t lds_needed(int op, int dtype, int64_t n, const ppx_config &c) {
    switch (op) {
        case PPX_OP_FFT: return fft_lds_bytes((int)n, c.problems_per_block, c.algo, c.radix);
        case PPX_OP_SCAN: return scan_lds_bytes((int)n, c.problems_per_block, c.elems_per_thread, dtype);
        default: return tridiag_lds_bytes((int)n, c, dtype);
    }
}

// Elements held in LDS per workgroup (the paper's S).
static int lds_elems(int op, int64_t n, const ppx_config &c) {
    switch (op) {
        case PPX_OP_FFT: return n <= c.radix ? 0 : (int)(c.problems_per_block * n);
        case PPX_OP_SCAN: {
            const int64_t T = n / c.elems_per_thread;  // threads per problem
            return T > kWave ? c.threads_per_block / kWave : 0;
        }
        default:
            if (tri_blk(c.algo, n, c.elems_per_thread)) return 2 * c.threads_per_block;  // lane slots, two sets
            if (tri_in_wave(c.algo)) return 0;
            return (int)((c.algo == PPX_TRI_PCR ? 2 : 1) * c.problems_per_block * n);
    }
}

void complete_config(int op, int, int64_t n, ppx_config &c) {
    if (c.radix == 0) c.radix = 2;
    if (c.elems_per_thread == 0 && c.threads_per_block > 0 && c.problems_per_block > 0)
        c.elems_per_thread = (int)(n * c.problems_per_block / c.threads_per_block);
    if (c.lds_elems == 0 && c.elems_per_thread > 0) c.lds_elems = lds_elems(op, n, c);
}

int validate_config(int op, int dtype, int64_t n, const ppx_config &c) {
    if (!is_valid_dtype(op, dtype)) return fail(PPX_EINVAL, "unsupported op / dtype");
    if (!is_pow2(n) || n < PPX_MIN_N || n > PPX_MAX_N) return fail(PPX_EINVAL, "n must be a power of two in [16, 16384]");
    const int L = c.threads_per_block, G = c.problems_per_block;
    if (!is_pow2(L) || L > kMaxThreadsPerBlock)
        return fail(PPX_ECONFIG, "threads_per_block must be a power of two <= 1024");
    if (!is_pow2(G) || G > kMaxProblemsPerBlock)
        return fail(PPX_ECONFIG, "problems_per_block must be a power of two <= 64");
    if (n * G % L != 0) return fail(PPX_ECONFIG, "threads_per_block must divide problems_per_block * n");
    const int64_t P = n * G / L;
    if (c.elems_per_thread != 0 && c.elems_per_thread != P)
        return fail(PPX_ECONFIG, "elems_per_thread must equal n * problems_per_block / threads_per_block");
    if (!is_pow2(P) || P < 2 || P > kMaxElemsPerThread)
        return fail(PPX_ECONFIG, "elements per thread must be a power of two in [2, 32]");
    if (P > n) return fail(PPX_ECONFIG, "a thread cannot hold elements of two problems (P > n)");
    ppx_config full = c;
    full.elems_per_thread = (int)P;
    switch (op) {
        case PPX_OP_FFT:
            if (c.radix != 2 && c.radix != 4 && c.radix != 8 && c.radix != 16)
                return fail(PPX_ECONFIG, "FFT radix must be 2, 4, 8 or 16");
            if (c.radix > P) return fail(PPX_ECONFIG, "FFT radix must not exceed elements per thread");
            if (L > fft_max_threads((int)P))
                return fail(PPX_ECONFIG, "FFT with 32 elements per thread allows at most 512 threads");
            if (c.algo < PPX_FFT_LDS || c.algo > PPX_FFT_LDS_SPLIT_PIPE)
                return fail(PPX_ECONFIG, "FFT algo must be PPX_FFT_LDS, _LDS_SPLIT, _LDS_PIPE or _LDS_SPLIT_PIPE");
            if ((c.algo & PPX_FFT_LDS_PIPE) && !fft_pipe_available(c.radix, (int)P))
                return fail(PPX_ECONFIG, "the persistent FFT variants need radix = elements per thread = 8 or 16");
            break;
        case PPX_OP_SCAN:
            if (c.radix != 0 && c.radix != 2) return fail(PPX_ECONFIG, "scan radix must be 2");
            if (c.algo < PPX_SCAN_KS || c.algo > PPX_SCAN_LF_PIPE)
                return fail(PPX_ECONFIG, "scan algo must be PPX_SCAN_KS, _LF, _KS_PIPE or _LF_PIPE");
            if (dtype == PPX_F64 && P > kScanF64MaxElems)
                return fail(PPX_ECONFIG, "float64 scan allows at most 16 elements per thread");
            break;
        case PPX_OP_TRIDIAG:
            if (c.radix != 0 && c.radix != 2) return fail(PPX_ECONFIG, "tridiagonal radix must be 2");
            if (tri_base(c.algo) < PPX_TRI_CR || tri_base(c.algo) > kTriMaxBase ||
                (c.algo & ~(PPX_TRI_PIPE | 7)) != 0)
                return fail(PPX_ECONFIG, "tridiagonal algo must be PPX_TRI_CR, _PCR, _CR_PCR, _CR_SHFL, _PCR_SHFL, _PCR_REG, _WM or _LF (the in-wave ones optionally | PPX_TRI_PIPE)");
            if ((c.algo & PPX_TRI_PIPE) &&
                (!tri_in_wave(c.algo) || P * (dtype == PPX_F64 ? 8 : 4) > kTriPipeMaxBytes))
                return fail(PPX_ECONFIG, "PPX_TRI_PIPE needs an in-wave variant and P * element size <= 128 bytes");
            if (tri_blk(c.algo, n, P)) {  // the hybrid across waves
                if (c.algo & PPX_TRI_PIPE) return fail(PPX_ECONFIG, "the multi-wave hybrid has no persistent form");
                if (n / P > kTriBlkMaxLanes) return fail(PPX_ECONFIG, "the hybrid needs n / P <= 1024");
                if (P > 16) return fail(PPX_ECONFIG, "the hybrid holds at most 16 equations per lane");
                if (L > tri_blk_max_threads(dtype == PPX_F64 ? 8 : 4, (int)P))
                    return fail(PPX_ECONFIG, "the multi-wave hybrid with 16 doubles per lane allows at most 512 threads");
            } else if (tri_in_wave(c.algo)) {
                if (n / P > kWave) return fail(PPX_ECONFIG, "shuffle variant needs n / P <= 64 (a system within a wave)");
                if (P > tri_wave_max_p(c.algo, dtype)) return fail(PPX_ECONFIG, "shuffle variant: too many elements per thread");
                if (L > kTriWaveMaxThreads) return fail(PPX_ECONFIG, "shuffle variant allows at most 256 threads");
            }
            break;
        default:
            return fail(PPX_EINVAL, "unknown op");
    }
    if (lds_needed(op, dtype, n, full) > lds_limit())
        return fail(PPX_ECONFIG, "configuration needs more LDS than a workgroup can allocate");
    if (c.lds_elems != 0 && c.lds_elems != lds_elems(op, n, full))
        return fail(PPX_ECONFIG, "lds_elems does not match the configuration (pass 0 to derive)");
    return PPX_OK;
}

int default_config(int op, int dtype, int64_t n, ppx_config &c) {
    if (!is_valid_dtype(op, dtype)) return fail(PPX_EINVAL, "unsupported op / dtype");
    if (!is_pow2(n) || n < PPX_MIN_N || n > PPX_MAX_N) return fail(PPX_EINVAL, "n must be a power of two in [16, 16384]");
    std::memset(&c, 0, sizeof c);
    c.radix = 2;
    c.problems_per_block = 1;
    c.threads_per_block = (int)(n / 2 < kMaxThreadsPerBlock ? n / 2 : kMaxThreadsPerBlock);
    c.algo = 0;
    if (op == PPX_OP_FFT && fft_lds_bytes((int)n, 1, PPX_FFT_LDS, c.radix) > lds_limit()) c.algo = PPX_FFT_LDS_SPLIT;
    complete_config(op, dtype, n, c);
    return validate_config(op, dtype, n, c);
}

// The search space enumerated by the tuners: r in {2,4,8,16} (FFT only),
// L in {64,...,1024}, G_b in {1,...,64}, and the algorithm variants of each
// operation; invalid points are dropped.
int enumerate_configs(int op, int dtype, int64_t n, ppx_config *out, int cap) {
    if (!is_valid_dtype(op, dtype)) return fail(PPX_EINVAL, "unsupported op / dtype");
    if (!is_pow2(n) || n < PPX_MIN_N || n > PPX_MAX_N) return fail(PPX_EINVAL, "n must be a power of two in [16, 16384]");
    static const int radices_fft[] = {2, 4, 8, 16};
    static const int radix_two[] = {2};
    const int *radices = op == PPX_OP_FFT ? radices_fft : radix_two;
    const int nr = op == PPX_OP_FFT ? 4 : 1;
    static const int algos_two[] = {0, 1, 2, 3};
    static const int algos_tri[] = {PPX_TRI_CR, PPX_TRI_PCR, PPX_TRI_CR_PCR, PPX_TRI_CR_SHFL, PPX_TRI_PCR_SHFL,
                                    PPX_TRI_PCR_REG, PPX_TRI_WM, PPX_TRI_LF, PPX_TRI_CR_PCR | PPX_TRI_PIPE,
                                    PPX_TRI_CR_SHFL | PPX_TRI_PIPE,
                                    PPX_TRI_PCR_SHFL | PPX_TRI_PIPE, PPX_TRI_PCR_REG | PPX_TRI_PIPE,
                                    PPX_TRI_WM | PPX_TRI_PIPE, PPX_TRI_LF | PPX_TRI_PIPE};
    const int *algos = op == PPX_OP_TRIDIAG ? algos_tri : algos_two;
    const int nalgo = op == PPX_OP_TRIDIAG ? (int)(sizeof algos_tri / sizeof algos_tri[0]) : 4;
    int count = 0;
    for (int ri = 0; ri < nr; ++ri)
        for (int L = 64; L <= 1024; L *= 2)
            for (int G = 1; G <= kMaxProblemsPerBlock; G *= 2)
                for (int ai = 0; ai < nalgo; ++ai) {
                    const int a = algos[ai];
                    ppx_config c{};
                    c.radix = radices[ri];
                    c.threads_per_block = L;
                    c.problems_per_block = G;
                    c.algo = a;
                    complete_config(op, dtype, n, c);
                    if (validate_config(op, dtype, n, c) != PPX_OK) continue;
                    // FFT: the split exchange only when it is needed or saves LDS
                    // (a single-stage transform uses no LDS at all).
                    if (op == PPX_OP_FFT && (a & PPX_FFT_LDS_SPLIT) && n <= c.radix) continue;
                    if (count < cap && out) out[count] = c;
                    ++count;
                }
    fail(PPX_OK, "");
    return count;
}

}  // namespace ppx
