// Batched tridiagonal solvers (Sec. III of arXiv:2310.16214): cyclic
// reduction (CR, Hockney) and parallel cyclic reduction (PCR, Hockney &
// Jesshope), float32 and float64, for gfx950.
//
// System: a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i, i < n, with the absent
// unknowns x_{-1} = x_n = 0; a_0 and c_{n-1} are never loaded (they are set to
// zero in LDS).  A workgroup of L threads solves G_b systems held in LDS as
// four arrays (a, b, c, d); its global loads and stores are flat, coalesced
// sweeps over the workgroup's G_b*n contiguous equations.
//
// CR.  Forward reduction, level l = 0..log2(n)-2 with s = 2^l: every equation
// i = 2s*j + 2s - 1 eliminates its neighbours i-s and i+s,
//     k1 = a_i / b_{i-s},  k2 = c_i / b_{i+s}   (k2 = 0 when i+s >= n)
//     a_i <- -a_{i-s} k1,  c_i <- -c_{i+s} k2
//     b_i <- b_i - c_{i-s} k1 - a_{i+s} k2,  d_i <- d_i - d_{i-s} k1 - d_{i+s} k2,
// leaving the 2x2 system of equations n/2-1 and n-1, solved directly; then
// back substitution, level l = log2(n)-2..0: every equation i = 2s*j + s - 1
// gets x_i = (d_i - a_i x_{i-s} - c_i x_{i+s}) / b_i (absent x are 0).  The
// solution overwrites d in LDS.
//
// PCR.  log2(n) steps, s = 2^l: every equation applies the same update using
// its neighbours at distance s (a missing neighbour is the identity row), read
// from one LDS buffer set and written to the other; after the last step every
// equation is decoupled and x_i = d_i / b_i.
#pragma once

#include <hip/hip_runtime.h>

#include "ppx_internal.h"

namespace ppx {

template <typename T>
__device__ __forceinline__ void tri_load(const T *a, const T *b, const T *c, const T *d, T *sa,
                                         T *sb, T *sc, T *sd, long long base, int total, int n) {
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int i = e & (n - 1);
        sa[e] = i == 0 ? T(0) : a[base + e];
        sb[e] = b[base + e];
        sc[e] = i == n - 1 ? T(0) : c[base + e];
        sd[e] = d[base + e];
    }
}

template <typename T>
__device__ void cr_solve(T *sa, T *sb, T *sc, T *sd, int log2n, int nsys) {
    const int n = 1 << log2n;
    const int L = blockDim.x;
    // forward reduction
    for (int ls = 0; ls < log2n - 1; ++ls) {
        const int s = 1 << ls;
        const int lper = log2n - ls - 1;  // log2 of active equations per system
        const int work = nsys << lper;
        for (int w = threadIdx.x; w < work; w += L) {
            const int sys = w >> lper;
            const int j = w & ((1 << lper) - 1);
            const int il = (j << (ls + 1)) + 2 * s - 1;  // local index
            const int i = sys * n + il;
            const bool hr = il + s < n;
            const T k1 = sa[i] / sb[i - s];
            T nb = sb[i] - sc[i - s] * k1;
            T nd = sd[i] - sd[i - s] * k1;
            T na = -sa[i - s] * k1;
            T nc = T(0);
            if (hr) {
                const T k2 = sc[i] / sb[i + s];
                nb -= sa[i + s] * k2;
                nd -= sd[i + s] * k2;
                nc = -sc[i + s] * k2;
            }
            sa[i] = na;
            sb[i] = nb;
            sc[i] = nc;
            sd[i] = nd;
        }
        __syncthreads();
    }
    // the remaining 2x2 system: equations n/2 - 1 and n - 1
    for (int sys = threadIdx.x; sys < nsys; sys += L) {
        const int i1 = sys * n + n / 2 - 1, i2 = sys * n + n - 1;
        const T b1 = sb[i1], c1 = sc[i1], d1 = sd[i1];
        const T a2 = sa[i2], b2 = sb[i2], d2 = sd[i2];
        const T det = b1 * b2 - c1 * a2;
        sd[i1] = (d1 * b2 - c1 * d2) / det;
        sd[i2] = (b1 * d2 - d1 * a2) / det;
    }
    __syncthreads();
    // back substitution
    for (int ls = log2n - 2; ls >= 0; --ls) {
        const int s = 1 << ls;
        const int lper = log2n - ls - 1;
        const int work = nsys << lper;
        for (int w = threadIdx.x; w < work; w += L) {
            const int sys = w >> lper;
            const int j = w & ((1 << lper) - 1);
            const int il = (j << (ls + 1)) + s - 1;
            const int i = sys * n + il;
            T r = sd[i];
            if (il >= s) r -= sa[i] * sd[i - s];
            if (il + s < n) r -= sc[i] * sd[i + s];
            sd[i] = r / sb[i];
        }
        __syncthreads();
    }
}

// Returns the LDS array that holds the solution.
template <typename T>
__device__ T *pcr_solve(T *sa, T *sb, T *sc, T *sd, T *ta, T *tb, T *tc, T *td, int log2n,
                        int total) {
    const int n = 1 << log2n;
    for (int ls = 0; ls < log2n; ++ls) {
        const int s = 1 << ls;
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int i = e & (n - 1);
            T na = T(0), nc = T(0);
            T nb = sb[e], nd = sd[e];
            if (i >= s) {
                const T k1 = sa[e] / sb[e - s];
                na = -sa[e - s] * k1;
                nb -= sc[e - s] * k1;
                nd -= sd[e - s] * k1;
            }
            if (i + s < n) {
                const T k2 = sc[e] / sb[e + s];
                nc = -sc[e + s] * k2;
                nb -= sa[e + s] * k2;
                nd -= sd[e + s] * k2;
            }
            ta[e] = na;
            tb[e] = nb;
            tc[e] = nc;
            td[e] = nd;
        }
        __syncthreads();
        T *t;
        t = sa; sa = ta; ta = t;
        t = sb; sb = tb; tb = t;
        t = sc; sc = tc; tc = t;
        t = sd; sd = td; td = t;
    }
    for (int e = threadIdx.x; e < total; e += blockDim.x) td[e] = sd[e] / sb[e];
    return td;  // read by the caller after a barrier
}

// One workgroup's share: systems [first, first + nsys); `smem` holds
// 4 * nsys * n (CR) or 8 * nsys * n (PCR) values.  Used by k_tridiag and by
// the fused kernel.
template <typename T, int ALGO>
__device__ __forceinline__ void tridiag_block(const T *a, const T *b, const T *c, const T *d, T *x,
                                              int log2n, long long first, int nsys, T *smem) {
    const int n = 1 << log2n;
    const int total = nsys * n;
    const long long base = first * n;
    const int cap = nsys * n;
    T *sa = smem, *sb = smem + cap, *sc = smem + 2 * cap, *sd = smem + 3 * cap;
    tri_load<T>(a, b, c, d, sa, sb, sc, sd, base, total, n);
    __syncthreads();
    const T *res;
    if constexpr (ALGO == PPX_TRI_CR) {
        cr_solve<T>(sa, sb, sc, sd, log2n, nsys);
        res = sd;
    } else {
        T *ta = smem + 4 * cap, *tb = smem + 5 * cap, *tc = smem + 6 * cap, *td = smem + 7 * cap;
        res = pcr_solve<T>(sa, sb, sc, sd, ta, tb, tc, td, log2n, total);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < total; e += blockDim.x) x[base + e] = res[e];
}

template <typename T, int ALGO>
__global__ __launch_bounds__(1024) void k_tridiag(const T *a, const T *b, const T *c, const T *d,
                                                  T *x, int log2n, long long batch, int gb) {
    extern __shared__ float4 smem_raw[];
    const long long first = (long long)blockIdx.x * gb;
    const int nsys = (int)min((long long)gb, batch - first);
    tridiag_block<T, ALGO>(a, b, c, d, x, log2n, first, nsys, reinterpret_cast<T *>(smem_raw));
}

}  // namespace ppx
