// Tridiagonal CR and PCR inside one wave (the paper's "shuffle" variant of
// Sec. V-A, where a problem small enough for one warp exchanges through
// shuffles instead of shared memory; on gfx950 the wave has 64 lanes, so the
// condition is n / P <= 64).
//
// Each system is owned by n / P consecutive lanes; lane t holds the P
// consecutive equations t*P .. t*P + P - 1 in registers (a, b, c, d).
//
// CR, forward level with stride s: equations i = 2s*m + 2s - 1 eliminate
// i - s and i + s (same update as the LDS kernel).  While 2s <= P the active
// equations and their left neighbours are in the lane's own registers and
// only i + s may be equation s - 1 of the next lane (one shuffle of four
// values).  From s = P on, the reduced system lives in each lane's last
// equation and the neighbours are the last equations of the lanes s/P away.
// The 2x2 system of equations n/2 - 1 and n - 1 is solved by both of their
// lanes; back substitution mirrors the levels, x overwriting d.
//
// PCR, step with stride s: every equation updates from its neighbours at
// distance s: for s < P the s nearest equations of the adjacent lanes come by
// shuffles, from s = P on each equation's neighbours are the same registers of
// the lanes s/P away.  After log2 n steps x_i = d_i / b_i.
//
// Out-of-system neighbours act as identity equations, which the row-index
// predicates implement; so several systems may share a wave and shuffles that
// cross a system boundary are ignored.  No LDS, no barriers.
#pragma once

#include <hip/hip_runtime.h>

#include "ppx_internal.h"

namespace ppx {

template <typename T>
__device__ __forceinline__ T shfl_up(T v, int d) { return __shfl_up(v, (unsigned)d, 64); }
template <typename T>
__device__ __forceinline__ T shfl_down(T v, int d) { return __shfl_down(v, (unsigned)d, 64); }

// Reciprocal: hardware estimate refined by Newton steps (two for double,
// one for float), instead of the IEEE division sequence.
__device__ __forceinline__ float rcp(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return r * (2.0f - x * r);
}
__device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = r * (2.0 - x * r);
    return r * (2.0 - x * r);
}

template <typename T, int P>
__device__ __forceinline__ void wave_load(const T *src, T (&v)[P]) {
    constexpr int V = 16 / sizeof(T);  // elements per 16-byte load
    if constexpr (P % V == 0) {
#pragma unroll
        for (int j = 0; j < P; j += V) {
            const int4 w = *reinterpret_cast<const int4 *>(src + j);
            T tmp[V];
            __builtin_memcpy(tmp, &w, 16);
#pragma unroll
            for (int k = 0; k < V; ++k) v[j + k] = tmp[k];
        }
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = src[j];
    }
}

template <typename T, int P>
__device__ __forceinline__ void wave_store(T *dst, const T (&v)[P]) {
    constexpr int V = 16 / sizeof(T);
    if constexpr (P % V == 0) {
#pragma unroll
        for (int j = 0; j < P; j += V) {
            T tmp[V];
#pragma unroll
            for (int k = 0; k < V; ++k) tmp[k] = v[j + k];
            int4 w;
            __builtin_memcpy(&w, tmp, 16);
            *reinterpret_cast<int4 *>(dst + j) = w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) dst[j] = v[j];
    }
}

// CR on the registers of one lane group; t = lane index within the system,
// lps = lanes per system, n = P * lps.
template <typename T, int P>
__device__ __forceinline__ void wave_cr(T (&a)[P], T (&b)[P], T (&c)[P], T (&d)[P], int t, int lps,
                                        int log2n) {
    const int n = P * lps;
    // ---- forward levels inside the lane (2s <= P)
#pragma unroll
    for (int s = 1; 2 * s <= P; s *= 2) {
        if (2 * s > n / 2) break;  // the last level leaves two equations
        // equation s - 1 of the next lane (current values)
        const T na = shfl_down(a[s - 1], 1), nb = shfl_down(b[s - 1], 1);
        const T nc = shfl_down(c[s - 1], 1), nd = shfl_down(d[s - 1], 1);
#pragma unroll
        for (int r = 2 * s - 1; r < P; r += 2 * s) {
            const T k1 = a[r] * rcp(b[r - s]);
            T nb_ = b[r] - c[r - s] * k1, nd_ = d[r] - d[r - s] * k1, na_ = -a[r - s] * k1, nc_ = T(0);
            const bool right_local = r + s < P;
            const bool has_right = right_local || t + 1 < lps;
            if (has_right) {
                const T ra = right_local ? a[(r + s) % P] : na;
                const T rb = right_local ? b[(r + s) % P] : nb;
                const T rc = right_local ? c[(r + s) % P] : nc;
                const T rd = right_local ? d[(r + s) % P] : nd;
                const T k2 = c[r] * rcp(rb);
                nb_ -= ra * k2;
                nd_ -= rd * k2;
                nc_ = -rc * k2;
            }
            a[r] = na_;
            b[r] = nb_;
            c[r] = nc_;
            d[r] = nd_;
        }
    }
    // ---- forward levels across lanes (s >= P): last equation of each lane
    for (int s = P; s <= n / 4; s *= 2) {
        const int dl = s / P;
        const T la = shfl_up(a[P - 1], dl), lb = shfl_up(b[P - 1], dl);
        const T lc = shfl_up(c[P - 1], dl), ld = shfl_up(d[P - 1], dl);
        const T ra = shfl_down(a[P - 1], dl), rb = shfl_down(b[P - 1], dl);
        const T rc = shfl_down(c[P - 1], dl), rd = shfl_down(d[P - 1], dl);
        if (((t + 1) & (2 * dl - 1)) == 0) {  // equation t*P + P - 1 is 2s*m + 2s - 1
            const T k1 = a[P - 1] * rcp(lb);
            T nb_ = b[P - 1] - lc * k1, nd_ = d[P - 1] - ld * k1, na_ = -la * k1, nc_ = T(0);
            if (t + dl < lps) {
                const T k2 = c[P - 1] * rcp(rb);
                nb_ -= ra * k2;
                nd_ -= rd * k2;
                nc_ = -rc * k2;
            }
            a[P - 1] = na_;
            b[P - 1] = nb_;
            c[P - 1] = nc_;
            d[P - 1] = nd_;
        }
    }
    // ---- the 2x2 system of equations n/2 - 1 and n - 1
    if (lps == 1) {
        const int i1 = n / 2 - 1, i2 = n - 1;
        const T det = b[i1 % P] * b[i2 % P] - c[i1 % P] * a[i2 % P];
        const T x1 = (d[i1 % P] * b[i2 % P] - c[i1 % P] * d[i2 % P]) * rcp(det);
        const T x2 = (b[i1 % P] * d[i2 % P] - d[i1 % P] * a[i2 % P]) * rcp(det);
        d[i1 % P] = x1;
        d[i2 % P] = x2;
    } else {
        const int h = lps / 2;  // lanes h-1 and lps-1 hold the two equations
        const T oa = shfl_down(a[P - 1], h), ob = shfl_down(b[P - 1], h);
        const T oc = shfl_down(c[P - 1], h), od = shfl_down(d[P - 1], h);
        const T ua = shfl_up(a[P - 1], h), ub = shfl_up(b[P - 1], h);
        const T uc = shfl_up(c[P - 1], h), ud = shfl_up(d[P - 1], h);
        if (t == h - 1) {  // row 1 here, row 2 from lane t + h
            const T det = b[P - 1] * ob - c[P - 1] * oa;
            d[P - 1] = (d[P - 1] * ob - c[P - 1] * od) * rcp(det);
        } else if (t == lps - 1) {  // row 2 here, row 1 from lane t - h
            const T det = ub * b[P - 1] - uc * a[P - 1];
            d[P - 1] = (ub * d[P - 1] - ud * a[P - 1]) * rcp(det);
        }
        (void)uc;
        (void)oc;
    }
    // ---- back substitution across lanes (s >= P)
    for (int s = n / 4; s >= P; s /= 2) {
        const int dl = s / P;
        const T xl = shfl_up(d[P - 1], dl), xr = shfl_down(d[P - 1], dl);
        if (((t + 1) & (2 * dl - 1)) == dl) {  // equation 2s*m + s - 1
            T r = d[P - 1];
            if (t - dl >= 0) r -= a[P - 1] * xl;
            if (t + dl < lps) r -= c[P - 1] * xr;
            d[P - 1] = r * rcp(b[P - 1]);
        }
    }
    // ---- back substitution inside the lane (s < P)
#pragma unroll
    for (int s = P / 2; s >= 1; s /= 2) {
        if (2 * s > n / 2) continue;
        const T xl = shfl_up(d[P - 1], 1);  // x of the previous lane's last equation
#pragma unroll
        for (int r = s - 1; r < P; r += 2 * s) {
            T v = d[r];
            if (r >= s) v -= a[r] * d[r - s];
            else if (t > 0) v -= a[r] * xl;
            if (r + s < P) v -= c[r] * d[r + s];  // always local: r + s <= P - 1
            d[r] = v * rcp(b[r]);
        }
    }
    (void)log2n;
}

// PCR update of one equation from its left (l*) and right (r*) neighbours;
// has_l / has_r false mean identity neighbours.
template <typename T>
__device__ __forceinline__ void pcr_update(T &a, T &b, T &c, T &d, T la, T lb, T lc, T ld, T ra, T rb,
                                           T rc, T rd, bool has_l, bool has_r) {
    T na = T(0), nc = T(0), nb = b, nd = d;
    if (has_l) {
        const T k1 = a * rcp(lb);
        na = -la * k1;
        nb -= lc * k1;
        nd -= ld * k1;
    }
    if (has_r) {
        const T k2 = c * rcp(rb);
        nc = -rc * k2;
        nb -= ra * k2;
        nd -= rd * k2;
    }
    a = na;
    b = nb;
    c = nc;
    d = nd;
}

// PCR steps with stride S < P, unrolled: the left neighbours of equations
// r < S are equations P - S + r of the previous lane, the right neighbours of
// r >= P - S equations r + S - P of the next lane (8 S shuffles per step).
template <typename T, int P, int S>
__device__ __forceinline__ void pcr_inlane_steps(T (&a)[P], T (&b)[P], T (&c)[P], T (&d)[P], int t,
                                                 int n) {
    if constexpr (S < P) {
        if (S >= n) return;
        T ua[S], ub[S], uc[S], ud[S], wa[S], wb[S], wc[S], wd[S];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            ua[k] = shfl_up(a[P - S + k], 1);
            ub[k] = shfl_up(b[P - S + k], 1);
            uc[k] = shfl_up(c[P - S + k], 1);
            ud[k] = shfl_up(d[P - S + k], 1);
            wa[k] = shfl_down(a[k], 1);
            wb[k] = shfl_down(b[k], 1);
            wc[k] = shfl_down(c[k], 1);
            wd[k] = shfl_down(d[k], 1);
        }
        T na[P], nb[P], nc[P], nd[P];
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const int i = t * P + r;
            na[r] = a[r];
            nb[r] = b[r];
            nc[r] = c[r];
            nd[r] = d[r];
            const T la = r >= S ? a[r - S] : ua[r % S], lb = r >= S ? b[r - S] : ub[r % S];
            const T lc = r >= S ? c[r - S] : uc[r % S], ld = r >= S ? d[r - S] : ud[r % S];
            const T ra = r + S < P ? a[(r + S) % P] : wa[(r + S) % S];
            const T rb = r + S < P ? b[(r + S) % P] : wb[(r + S) % S];
            const T rc = r + S < P ? c[(r + S) % P] : wc[(r + S) % S];
            const T rd = r + S < P ? d[(r + S) % P] : wd[(r + S) % S];
            pcr_update(na[r], nb[r], nc[r], nd[r], la, lb, lc, ld, ra, rb, rc, rd, i - S >= 0, i + S < n);
        }
#pragma unroll
        for (int r = 0; r < P; ++r) {
            a[r] = na[r];
            b[r] = nb[r];
            c[r] = nc[r];
            d[r] = nd[r];
        }
        pcr_inlane_steps<T, P, 2 * S>(a, b, c, d, t, n);
    }
}

// PCR on the registers of one lane group.
template <typename T, int P>
__device__ __forceinline__ void wave_pcr(T (&a)[P], T (&b)[P], T (&c)[P], T (&d)[P], int t, int lps,
                                         int log2n) {
    const int n = P * lps;
    pcr_inlane_steps<T, P, 1>(a, b, c, d, t, n);
    // strides s >= P: the neighbours are the same registers of the lanes s/P
    // away; each equation only needs its own old values and the shuffled
    // ones, so the update is in place (all lanes step through r together)
    for (int s = P; s < n; s *= 2) {
        const int dl = s / P;
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const T la = shfl_up(a[r], dl), lb = shfl_up(b[r], dl);
            const T lc = shfl_up(c[r], dl), ld = shfl_up(d[r], dl);
            const T ra = shfl_down(a[r], dl), rb = shfl_down(b[r], dl);
            const T rc = shfl_down(c[r], dl), rd = shfl_down(d[r], dl);
            pcr_update(a[r], b[r], c[r], d[r], la, lb, lc, ld, ra, rb, rc, rd, t - dl >= 0, t + dl < lps);
        }
    }
#pragma unroll
    for (int r = 0; r < P; ++r) d[r] = d[r] * rcp(b[r]);
    (void)log2n;
}

// One workgroup's share: systems [first, first + nsys) of size n = P * lps,
// lps = n / P <= 64 lanes each; every lane owns P equations.
template <typename T, int ALGO, int P>
__device__ __forceinline__ void tridiag_wave_block(const T *A, const T *B, const T *C, const T *D,
                                                   T *X, int log2n, long long first, int nsys) {
    const int n = 1 << log2n;
    const int lps = n / P;
    const int sys_local = threadIdx.x / lps;
    const int t = threadIdx.x % lps;
    const bool active = sys_local < nsys;
    const long long base = (first + sys_local) * n + (long long)t * P;
    T a[P], b[P], c[P], d[P];
    if (active) {
        wave_load<T, P>(A + base, a);
        wave_load<T, P>(B + base, b);
        wave_load<T, P>(C + base, c);
        wave_load<T, P>(D + base, d);
        if (t == 0) a[0] = T(0);            // multiplies the absent x_{-1}
        if (t == lps - 1) c[P - 1] = T(0);  // multiplies the absent x_n
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            a[j] = T(0);
            b[j] = T(1);
            c[j] = T(0);
            d[j] = T(0);
        }
    }
    if constexpr (ALGO == PPX_TRI_CR_SHFL) wave_cr<T, P>(a, b, c, d, t, lps, log2n);
    else wave_pcr<T, P>(a, b, c, d, t, lps, log2n);
    if (active) wave_store<T, P>(X + base, d);
}

template <typename T, int ALGO, int P>
__global__ __launch_bounds__(256) void k_tridiag_wave(const T *a, const T *b, const T *c, const T *d,
                                                      T *x, int log2n, long long batch, int gb) {
    const long long first = (long long)blockIdx.x * gb;
    const int nsys = (int)min((long long)gb, batch - first);
    tridiag_wave_block<T, ALGO, P>(a, b, c, d, x, log2n, first, nsys);
}

}  // namespace ppx
