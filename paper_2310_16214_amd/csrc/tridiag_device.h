// Batched tridiagonal solvers (Sec. III of arXiv:2310.16214): cyclic
// reduction (CR, Hockney) and parallel cyclic reduction (PCR, Hockney &
// Jesshope), float32 and float64, for gfx950.
//
// System: a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i, i < n, with the absent
// unknowns x_{-1} = x_n = 0; a_0 and c_{n-1} are replaced by zero at load.
//
// Every equation is kept scaled to unit diagonal: row i is divided by b_i at
// load and again after each elimination.  Row scaling changes neither the
// solution nor which unknowns CR and PCR eliminate at each level; it means a
// neighbour row contributes three values (a, c, d) instead of four, an
// elimination needs one reciprocal instead of two divisions, back substitution
// needs none, and after the last PCR step x_i = d_i.  With unit-diagonal rows
// l = (la, 1, lc, ld) at i - s and r = (ra, 1, rc, rd) at i + s, the update of
// row i = (a, 1, c, d) (the paper's k1 = a_i / b_{i-s} and k2 = c_i / b_{i+s}
// are then just a and c) is
//     b' = 1 - lc a - ra c
//     (a, c, d) <- (-la a, -rc c, d - ld a - rd c) / b'
// and an absent neighbour is the identity row, i.e. zeros.
//
// CR.  Forward reduction, level l = 0..log2(n)-2 with s = 2^l: every equation
// i = 2s*j + 2s - 1 eliminates its neighbours i-s and i+s, leaving the 2x2
// system of equations n/2-1 and n-1, solved directly; then back substitution,
// level l = log2(n)-2..0: every equation i = 2s*j + s - 1 gets
// x_i = d_i - a_i x_{i-s} - c_i x_{i+s} (absent x are 0).
//
// PCR.  log2(n) steps, s = 2^l: every equation applies the update with its
// neighbours at distance s, read from one buffer set and written to the other.
//
// The LDS kernels here hold a workgroup's G_b systems as three arrays (a, c,
// d; PCR: two sets); global loads and stores are flat, coalesced sweeps over
// the workgroup's G_b*n contiguous equations.
#pragma once

#include <hip/hip_runtime.h>

#include "ppx_internal.h"

namespace ppx {

// Reciprocal instead of the IEEE division sequence: for float the hardware
// instruction (accurate to 1 ulp), for double its estimate refined by two
// Newton steps.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = r * (2.0 - x * r);
    return r * (2.0 - x * r);
}

// The unit-diagonal elimination of row (a, 1, c, d) with its neighbour rows
// (la, 1, lc, ld) and (ra, 1, rc, rd); zeros stand for an absent neighbour.
template <typename T>
__device__ __forceinline__ void unit_eliminate(T &a, T &c, T &d, T la, T lc, T ld, T ra, T rc, T rd) {
    const T r = rcp(T(1) - lc * a - ra * c);
    const T nd = (d - ld * a - rd * c) * r;
    a = -(la * a) * r;
    c = -(rc * c) * r;
    d = nd;
}

template <typename T>
__device__ __forceinline__ void tri_load(const T *a, const T *b, const T *c, const T *d, T *sa,
                                         T *sc, T *sd, long long base, int total, int n) {
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int i = e & (n - 1);
        const T r = rcp(b[base + e]);
        const T av = a[base + e], cv = c[base + e];
        sa[e] = i == 0 ? T(0) : av * r;
        sc[e] = i == n - 1 ? T(0) : cv * r;
        sd[e] = d[base + e] * r;
    }
}

template <typename T>
__device__ void cr_solve(T *sa, T *sc, T *sd, int log2n, int nsys) {
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
            T ra = T(0), rc = T(0), rd = T(0);
            if (il + s < n) {
                ra = sa[i + s];
                rc = sc[i + s];
                rd = sd[i + s];
            }
            T a = sa[i], c = sc[i], d = sd[i];
            unit_eliminate(a, c, d, sa[i - s], sc[i - s], sd[i - s], ra, rc, rd);
            sa[i] = a;
            sc[i] = c;
            sd[i] = d;
        }
        __syncthreads();
    }
    // the remaining 2x2 system: equations n/2 - 1 and n - 1
    for (int sys = threadIdx.x; sys < nsys; sys += L) {
        const int i1 = sys * n + n / 2 - 1, i2 = sys * n + n - 1;
        const T c1 = sc[i1], d1 = sd[i1], a2 = sa[i2], d2 = sd[i2];
        const T r = rcp(T(1) - c1 * a2);
        sd[i1] = (d1 - c1 * d2) * r;
        sd[i2] = (d2 - a2 * d1) * r;
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
            T x = sd[i];
            if (il >= s) x -= sa[i] * sd[i - s];
            if (il + s < n) x -= sc[i] * sd[i + s];
            sd[i] = x;
        }
        __syncthreads();
    }
}

// Returns the LDS array that holds the solution (after the final barrier).
template <typename T>
__device__ T *pcr_solve(T *sa, T *sc, T *sd, T *ta, T *tc, T *td, int log2n, int total) {
    const int n = 1 << log2n;
    for (int ls = 0; ls < log2n; ++ls) {
        const int s = 1 << ls;
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int i = e & (n - 1);
            T la = T(0), lc = T(0), ld = T(0), ra = T(0), rc = T(0), rd = T(0);
            if (i >= s) {
                la = sa[e - s];
                lc = sc[e - s];
                ld = sd[e - s];
            }
            if (i + s < n) {
                ra = sa[e + s];
                rc = sc[e + s];
                rd = sd[e + s];
            }
            T a = sa[e], c = sc[e], d = sd[e];
            unit_eliminate(a, c, d, la, lc, ld, ra, rc, rd);
            ta[e] = a;
            tc[e] = c;
            td[e] = d;
        }
        __syncthreads();
        T *t;
        t = sa; sa = ta; ta = t;
        t = sc; sc = tc; tc = t;
        t = sd; sd = td; td = t;
    }
    return sd;
}

// LDS values per system: three arrays for CR, two sets of three for PCR.
constexpr int tri_lds_arrays(int algo) { return algo == PPX_TRI_PCR ? 6 : 3; }

// One workgroup's share: systems [first, first + nsys); `smem` holds
// tri_lds_arrays(ALGO) * nsys * n values.  Used by k_tridiag and by the fused
// kernel.
template <typename T, int ALGO>
__device__ __forceinline__ void tridiag_block(const T *a, const T *b, const T *c, const T *d, T *x,
                                              int log2n, long long first, int nsys, T *smem) {
    const int n = 1 << log2n;
    const int total = nsys * n;
    const long long base = first * n;
    T *sa = smem, *sc = smem + total, *sd = smem + 2 * total;
    tri_load<T>(a, b, c, d, sa, sc, sd, base, total, n);
    __syncthreads();
    const T *res;
    if constexpr (ALGO == PPX_TRI_CR) {
        cr_solve<T>(sa, sc, sd, log2n, nsys);
        res = sd;
    } else {
        res = pcr_solve<T>(sa, sc, sd, smem + 3 * total, smem + 4 * total, smem + 5 * total, log2n,
                           total);
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
