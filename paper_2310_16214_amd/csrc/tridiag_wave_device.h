// Tridiagonal CR, PCR, Wang & Mou and Ladner-Fischer solvers inside one wave
// (the paper's "shuffle" variant of Sec. V-A, where a problem small enough for
// one warp exchanges through shuffles instead of shared memory; on gfx950 the wave has 64 lanes, so the
// condition is n / P <= 64).  Rows are kept at unit diagonal and eliminated by
// unit_eliminate, as in the LDS kernels of tridiag_device.h.
//
// Each system is owned by n / P consecutive lanes; lane t holds the P
// consecutive equations t*P .. t*P + P - 1 in registers (a, c, d after the
// scaling at load).
//
// CR, forward level with stride s: equations i = 2s*m + 2s - 1 eliminate
// i - s and i + s.  While 2s <= P the active equations and their left
// neighbours are in the lane's own registers and only i + s may be equation
// s - 1 of the next lane (one shuffle of three values).  From s = P on, the
// reduced system lives in each lane's last equation and the neighbours are the
// last equations of the lanes s/P away.  The 2x2 system of equations n/2 - 1
// and n - 1 is solved by both of their lanes; back substitution mirrors the
// levels, x overwriting d.
//
// PCR, step with stride s: every equation updates from its neighbours at
// distance s: for s < P the s nearest equations of the adjacent lanes come by
// shuffles, from s = P on each equation's neighbours are the same registers of
// the lanes s/P away.  After log2 n steps x_i = d_i.
//
// Neighbours outside the system are identity rows.  CR replaces them by zeros
// explicitly.  PCR shuffles within the system's lanes only, so a lane whose
// neighbour lies outside the system receives one of its own (finite) values,
// and that value is multiplied by an exact zero: before the step with stride
// s, a_i = 0 for every i < s and c_i = 0 for every i >= n - s (true at load,
// where a_0 = c_{n-1} = 0, and kept by the update, whose new a_i is a product
// with a_{i-s} and a_i, and new c_i one with c_{i+s} and c_i).  Several
// systems may thus share a wave and no value crosses between them.  No LDS,
// no barriers.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"
#include "ppx_internal.h"
#include "tridiag_device.h"

namespace ppx {

template <typename T>
__device__ __forceinline__ T shfl_up(T v, int d) { return __shfl_up(v, (unsigned)d, 64); }
template <typename T>
__device__ __forceinline__ T shfl_down(T v, int d) { return __shfl_down(v, (unsigned)d, 64); }
// Shuffles confined to a system's lps lanes: a lane whose source would lie
// outside its system gets its own value back.
template <typename T>
__device__ __forceinline__ T sys_up(T v, int d, int lps) { return __shfl_up(v, (unsigned)d, lps); }
template <typename T>
__device__ __forceinline__ T sys_down(T v, int d, int lps) { return __shfl_down(v, (unsigned)d, lps); }

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

// Store policy of the solution x: non-temporal for float32 where a lane
// writes at most 32 bytes, the default otherwise.  On a plain copy with the
// solvers' traffic (four 16 MiB inputs read, one written) the hint takes the
// call from 19 to 16 us at 16 or 32 bytes per lane and makes it slower at 64
// (21 us); on the float32 solvers with P <= 8 it took 11-13% off the call,
// on float64 it measured neutral (within 1.5%), so float64 keeps the default.
template <typename T, int P>
constexpr bool tri_nt_stores() { return sizeof(T) == 4 && P * (int)sizeof(T) <= 32; }

template <typename T, int P>
__device__ __forceinline__ void wave_store(T *dst, const T (&v)[P]) {
    constexpr int V = 16 / sizeof(T);
    if constexpr (P % V == 0) {
#pragma unroll
        for (int j = 0; j < P; j += V) {
            T tmp[V];
#pragma unroll
            for (int k = 0; k < V; ++k) tmp[k] = v[j + k];
            u32x4 w;
            __builtin_memcpy(&w, tmp, 16);
            if constexpr (tri_nt_stores<T, P>()) store_nt(reinterpret_cast<u32x4 *>(dst + j), w);
            else *reinterpret_cast<u32x4 *>(dst + j) = w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) dst[j] = v[j];
    }
}

// CR forward levels inside the lane (2s <= P, and 2s <= n/4 so that the last
// level leaves two equations): equation r = 2s*m + 2s - 1 eliminates r - s and
// r + s; only the right neighbour of the lane's last active equation can be
// equation s - 1 of the next lane (one shuffle of three values).  After them
// each lane's last equation couples the last equations of the lanes beside it.
template <typename T, int P>
__device__ __forceinline__ void cr_inlane_forward(T (&a)[P], T (&c)[P], T (&d)[P], int t, int lps) {
    const int n = P * lps;
    const bool last_lane = t + 1 == lps;
#pragma unroll
    for (int s = 1; 2 * s <= P; s *= 2) {
        if (2 * s > n / 2) break;  // the last level leaves two equations
        // equation s - 1 of the next lane: right neighbour of equation P - 1
        T na = shfl_down(a[s - 1], 1), nc = shfl_down(c[s - 1], 1), nd = shfl_down(d[s - 1], 1);
        if (last_lane) na = nc = nd = T(0);
#pragma unroll
        for (int r = 2 * s - 1; r < P; r += 2 * s) {
            const bool local = r + s < P;
            unit_eliminate(a[r], c[r], d[r], a[r - s], c[r - s], d[r - s], local ? a[(r + s) % P] : na,
                           local ? c[(r + s) % P] : nc, local ? d[(r + s) % P] : nd);
        }
    }
}

// CR back substitution inside the lane (s < P), once every lane's last
// unknown is in d[P - 1]: equation r = 2s*m + s - 1 gets x_r = d_r - a_r
// x_{r-s} - c_r x_{r+s}, where x_{r-s} for the lane's first such equation is
// the previous lane's last unknown.
template <typename T, int P>
__device__ __forceinline__ void cr_inlane_backward(T (&a)[P], T (&c)[P], T (&d)[P], int t, int lps) {
    const int n = P * lps;
#pragma unroll
    for (int s = P / 2; s >= 1; s /= 2) {
        if (2 * s > n / 2) continue;
        const T xl = shfl_up(d[P - 1], 1);  // x of the previous lane's last equation
#pragma unroll
        for (int r = s - 1; r < P; r += 2 * s) {
            T x = d[r];
            if (r >= s) x -= a[r] * d[r - s];
            else if (t > 0) x -= a[r] * xl;
            x -= c[r] * d[r + s];  // r + s <= P - 1: always local
            d[r] = x;
        }
    }
}

// The 2x2 system of one lane's equations P/2 - 1 and P - 1 (a system held by
// a single lane, after the in-lane levels).
template <typename T, int P>
__device__ __forceinline__ void cr_solve_pair_inlane(T (&a)[P], T (&c)[P], T (&d)[P]) {
    constexpr int i1 = P / 2 - 1, i2 = P - 1;
    const T r = rcp(T(1) - c[i1] * a[i2]);
    const T x1 = (d[i1] - c[i1] * d[i2]) * r;
    const T x2 = (d[i2] - a[i2] * d[i1]) * r;
    d[i1] = x1;
    d[i2] = x2;
}

// CR on the registers of one lane group; t = lane index within the system,
// lps = lanes per system, n = P * lps.
template <typename T, int P>
__device__ __forceinline__ void wave_cr(T (&a)[P], T (&c)[P], T (&d)[P], int t, int lps) {
    const int n = P * lps;
    const bool last_lane = t + 1 == lps;
    cr_inlane_forward<T, P>(a, c, d, t, lps);
    // ---- forward levels across lanes (s >= P): last equation of each lane
    for (int s = P; s <= n / 4; s *= 2) {
        const int dl = s / P;
        const T la = shfl_up(a[P - 1], dl), lc = shfl_up(c[P - 1], dl), ld = shfl_up(d[P - 1], dl);
        T ra = shfl_down(a[P - 1], dl), rc = shfl_down(c[P - 1], dl), rd = shfl_down(d[P - 1], dl);
        if (t + dl >= lps) ra = rc = rd = T(0);
        // equation t*P + P - 1 is 2s*m + 2s - 1; its left neighbour exists
        if (((t + 1) & (2 * dl - 1)) == 0) unit_eliminate(a[P - 1], c[P - 1], d[P - 1], la, lc, ld, ra, rc, rd);
    }
    // ---- the 2x2 system of equations n/2 - 1 and n - 1
    if (lps == 1) {
        cr_solve_pair_inlane<T, P>(a, c, d);
    } else {
        const int h = lps / 2;  // lanes h-1 and lps-1 hold the two equations
        const T oa = shfl_down(a[P - 1], h), od = shfl_down(d[P - 1], h);
        const T uc = shfl_up(c[P - 1], h), ud = shfl_up(d[P - 1], h);
        if (t == h - 1) {  // row 1 here, row 2 from lane t + h
            d[P - 1] = (d[P - 1] - c[P - 1] * od) * rcp(T(1) - c[P - 1] * oa);
        } else if (last_lane) {  // row 2 here, row 1 from lane t - h
            d[P - 1] = (d[P - 1] - a[P - 1] * ud) * rcp(T(1) - uc * a[P - 1]);
        }
    }
    // ---- back substitution across lanes (s >= P)
    for (int s = n / 4; s >= P; s /= 2) {
        const int dl = s / P;
        const T xl = shfl_up(d[P - 1], dl), xr = shfl_down(d[P - 1], dl);
        if (((t + 1) & (2 * dl - 1)) == dl) {  // equation 2s*m + s - 1
            T x = d[P - 1];
            if (t - dl >= 0) x -= a[P - 1] * xl;
            if (t + dl < lps) x -= c[P - 1] * xr;
            d[P - 1] = x;
        }
    }
    cr_inlane_backward<T, P>(a, c, d, t, lps);
}

// CR -> PCR hybrid (PPX_TRI_CR_PCR): the CR levels inside the lane reduce
// each lane's P equations to its last one; PCR then solves that reduced
// system of lps equations (one per lane, stride P in the original indices)
// in log2(lps) steps, every lane active, with shuffles confined to the
// system's lanes (an out-of-system neighbour meets an exact zero coefficient,
// as in wave_pcr: lane 0's reduced a and the last lane's reduced c are
// products with the zeroed boundary coefficients); back substitution inside
// the lane then recovers the other equations.  Work per lane: P - 1
// eliminations, log2(lps) eliminations and P - 1 substitutions, against
// PCR's P log2(n) eliminations and CR's 2 log2(lps) cross-lane levels with
// most lanes idle.
template <typename T, int P>
__device__ __forceinline__ void wave_cr_pcr(T (&a)[P], T (&c)[P], T (&d)[P], int t, int lps) {
    cr_inlane_forward<T, P>(a, c, d, t, lps);
    if (lps == 1) {
        cr_solve_pair_inlane<T, P>(a, c, d);
    } else {
        for (int dl = 1; dl < lps; dl *= 2) {
            const T la = sys_up(a[P - 1], dl, lps), lc = sys_up(c[P - 1], dl, lps), ld = sys_up(d[P - 1], dl, lps);
            const T ra = sys_down(a[P - 1], dl, lps), rc = sys_down(c[P - 1], dl, lps),
                    rd = sys_down(d[P - 1], dl, lps);
            unit_eliminate(a[P - 1], c[P - 1], d[P - 1], la, lc, ld, ra, rc, rd);
        }
    }
    cr_inlane_backward<T, P>(a, c, d, t, lps);
}

// PCR steps with stride S < P, unrolled: the left neighbours of equations
// r < S are equations P - S + r of the previous lane, the right neighbours of
// r >= P - S equations r + S - P of the next lane (6 S shuffles per step).
template <typename T, int P, int S>
__device__ __forceinline__ void pcr_inlane_steps(T (&a)[P], T (&c)[P], T (&d)[P], int lps) {
    if constexpr (S < P) {
        T ua[S], uc[S], ud[S], wa[S], wc[S], wd[S];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            ua[k] = sys_up(a[P - S + k], 1, lps);
            uc[k] = sys_up(c[P - S + k], 1, lps);
            ud[k] = sys_up(d[P - S + k], 1, lps);
            wa[k] = sys_down(a[k], 1, lps);
            wc[k] = sys_down(c[k], 1, lps);
            wd[k] = sys_down(d[k], 1, lps);
        }
        T na[P], nc[P], nd[P];
#pragma unroll
        for (int r = 0; r < P; ++r) {
            na[r] = a[r];
            nc[r] = c[r];
            nd[r] = d[r];
            const bool lloc = r >= S, rloc = r + S < P;
            unit_eliminate(na[r], nc[r], nd[r], lloc ? a[(r + P - S) % P] : ua[r % S],
                           lloc ? c[(r + P - S) % P] : uc[r % S], lloc ? d[(r + P - S) % P] : ud[r % S],
                           rloc ? a[(r + S) % P] : wa[(r + S) % S], rloc ? c[(r + S) % P] : wc[(r + S) % S],
                           rloc ? d[(r + S) % P] : wd[(r + S) % S]);
        }
#pragma unroll
        for (int r = 0; r < P; ++r) {
            a[r] = na[r];
            c[r] = nc[r];
            d[r] = nd[r];
        }
        pcr_inlane_steps<T, P, 2 * S>(a, c, d, lps);
    }
}

// PCR on the registers of one lane group.
template <typename T, int P>
__device__ __forceinline__ void wave_pcr(T (&a)[P], T (&c)[P], T (&d)[P], int lps) {
    const int n = P * lps;
    pcr_inlane_steps<T, P, 1>(a, c, d, lps);
    // strides s >= P: the neighbours are the same registers of the lanes s/P
    // away; each equation only needs its own old values and the shuffled
    // ones, so the update is in place (all lanes step through r together)
    for (int s = P; s < n; s *= 2) {
        const int dl = s / P;
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const T la = sys_up(a[r], dl, lps), lc = sys_up(c[r], dl, lps), ld = sys_up(d[r], dl, lps);
            const T ra = sys_down(a[r], dl, lps), rc = sys_down(c[r], dl, lps), rd = sys_down(d[r], dl, lps);
            unit_eliminate(a[r], c[r], d[r], la, lc, ld, ra, rc, rd);
            // 16 doubles per lane: keep the scheduler from hoisting every
            // row's shuffles (register pressure would halve the occupancy)
            if constexpr (P * sizeof(T) >= 128)
                if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// ---- PCR with the cross-lane exchange through LDS (PPX_TRI_PCR_REG)
//
// Same steps as wave_pcr, but for strides s >= P the lanes exchange through a
// per-wave LDS buffer instead of shuffles: a shuffle moves 4 bytes per lane
// through the LDS crossbar, while 16-byte LDS stores and loads move four times
// as much per instruction.  Per chunk of K registers, every lane stores its
// (a, c, d) chunk and loads the chunks of the lanes dl to either side (its own
// at the system's ends, which meet exact-zero coefficients as with the
// confined shuffles).  A wave's LDS instructions execute in issue order, so
// the loads see the stores before them and finish before the next chunk's
// stores; the fences only keep the compiler from reordering them.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A lane's K values as words of 16 bytes (8 when K * sizeof(T) = 8), word w
// of lane l at index w * 64 + l: each access instruction covers 64
// consecutive words.
template <typename T, int K>
struct XWords {
    static constexpr int bytes = K * (int)sizeof(T);
    static constexpr int wb = bytes >= 16 ? 16 : bytes;
    static constexpr int nw = bytes / wb;
    static constexpr int per = wb / (int)sizeof(T);
    using W = typename std::conditional<wb == 16, int4, int2>::type;
};

template <typename T, int K>
__device__ __forceinline__ void xstore(T *buf, int lane, const T *v) {
    using X = XWords<T, K>;
    typename X::W *w = reinterpret_cast<typename X::W *>(buf);
#pragma unroll
    for (int k = 0; k < X::nw; ++k) {
        typename X::W x;
        __builtin_memcpy(&x, v + k * X::per, X::wb);
        w[k * 64 + lane] = x;
    }
}

template <typename T, int K>
__device__ __forceinline__ void xload(const T *buf, int lane, T *v) {
    using X = XWords<T, K>;
    const typename X::W *w = reinterpret_cast<const typename X::W *>(buf);
#pragma unroll
    for (int k = 0; k < X::nw; ++k) {
        const typename X::W x = w[k * 64 + lane];
        __builtin_memcpy(v + k * X::per, &x, X::wb);
    }
}

// xb: this wave's 3 * 64 * K values of LDS.
template <typename T, int P>
__device__ __forceinline__ void wave_pcr_reg(T (&a)[P], T (&c)[P], T (&d)[P], int t, int lps, T *xb) {
    constexpr int K = P < 4 ? P : 4;
    constexpr int PL = 64 * K;
    const int n = P * lps;
    const int lane = threadIdx.x & 63;
    pcr_inlane_steps<T, P, 1>(a, c, d, lps);
    for (int s = P; s < n; s *= 2) {
        const int dl = s / P;
        const int ll = t >= dl ? lane - dl : lane;
        const int rl = t + dl < lps ? lane + dl : lane;
#pragma unroll
        for (int r0 = 0; r0 < P; r0 += K) {
            xstore<T, K>(xb, lane, a + r0);
            xstore<T, K>(xb + PL, lane, c + r0);
            xstore<T, K>(xb + 2 * PL, lane, d + r0);
            wave_lds_order();
            T la[K], lc[K], ld[K], ra[K], rc[K], rd[K];
            xload<T, K>(xb, ll, la);
            xload<T, K>(xb + PL, ll, lc);
            xload<T, K>(xb + 2 * PL, ll, ld);
            xload<T, K>(xb, rl, ra);
            xload<T, K>(xb + PL, rl, rc);
            xload<T, K>(xb + 2 * PL, rl, rd);
            wave_lds_order();
#pragma unroll
            for (int k = 0; k < K; ++k)
                unit_eliminate(a[r0 + k], c[r0 + k], d[r0 + k], la[k], lc[k], ld[k], ra[k], rc[k], rd[k]);
        }
    }
}

// ---- Wang & Mou divide and conquer (PPX_TRI_WM)
//
// Every equation i of a block [s, e] of consecutive equations is kept solved
// for its own unknown in terms of the two unknowns just outside the block:
//     x_i = d_i - a_i x_{s-1} - c_i x_{e+1}
// (a unit-diagonal row is this form for the block [i, i]).  Two adjacent
// blocks L = [s, m] and R = [m+1, e] merge by solving the last equation of L
// and the first of R for x_m and x_{m+1} (pivot 1 - c_m a_{m+1}), which gives
// both in terms of x_{s-1} and x_{e+1}; every equation of L then replaces its
// x_{m+1} term, every equation of R its x_m term.  Blocks double at each level:
// after log2 n levels the block is the whole system, whose outer unknowns are
// absent, and x_i = d_i.  The first log2 P levels merge a lane's own P
// equations (the radix-P node); each further level needs only the two
// boundary equations, broadcast to the lanes of the merging pair of lane
// blocks.  A block that starts at equation 0 keeps a = 0 and one that ends at
// n - 1 keeps c = 0 (the pivot terms that would change them are products with
// those zeros), so several systems may share a wave: no merge crosses a
// system, whose lanes form an aligned group of lps lanes.

// The values the two halves apply: x_{m+1} = dn - an X - cn Y (for L) and
// x_m = dm - am X - cm Y (for R), X = x_{s-1}, Y = x_{e+1}.
template <typename T>
struct WmJoin {
    T an, cn, dn, am, cm, dm;
};

template <typename T>
__device__ __forceinline__ WmJoin<T> wm_join(T aL, T cL, T dL, T aR, T cR, T dR) {
    const T r = rcp(T(1) - cL * aR);
    WmJoin<T> j;
    j.dn = (dR - aR * dL) * r;
    j.an = -(aR * aL) * r;
    j.cn = cR * r;
    j.dm = (dL - cL * dR) * r;
    j.am = aL * r;
    j.cm = -(cL * cR) * r;
    return j;
}

// Equation of L: substitute x_{m+1}.
template <typename T>
__device__ __forceinline__ void wm_left(T &a, T &c, T &d, const WmJoin<T> &j) {
    d -= c * j.dn;
    a -= c * j.an;
    c = -(c * j.cn);
}

// Equation of R: substitute x_m.
template <typename T>
__device__ __forceinline__ void wm_right(T &a, T &c, T &d, const WmJoin<T> &j) {
    d -= a * j.dm;
    c -= a * j.cm;
    a = -(a * j.am);
}

// The levels inside a lane: blocks of s equations merge in pairs, s < P.
template <typename T, int P>
__device__ __forceinline__ void wm_inlane(T (&a)[P], T (&c)[P], T (&d)[P]) {
#pragma unroll
    for (int s = 1; s < P; s *= 2) {
#pragma unroll
        for (int b = 0; b < P; b += 2 * s) {
            const int m = b + s - 1;
            const WmJoin<T> j = wm_join(a[m], c[m], d[m], a[m + 1], c[m + 1], d[m + 1]);
#pragma unroll
            for (int i = b; i <= m; ++i) wm_left(a[i], c[i], d[i], j);
#pragma unroll
            for (int i = m + 1; i < b + 2 * s; ++i) wm_right(a[i], c[i], d[i], j);
        }
    }
}

// Lane level K: blocks of 2^K lanes merge in pairs.  The last equation of the
// left block sits in lane (lane & ~(2^(K+1) - 1)) + 2^K - 1, the first of the
// right block in the next lane; swizzle broadcasts within 32-lane halves for
// K < 5, lanes 31 and 32 for K = 5 (one system per wave).  Branch-free: a
// lane of the left block substitutes x_{m+1} (through c), one of the right
// block x_m (through a).
template <typename T, int P, int K>
__device__ __forceinline__ void wm_lane_level(T (&a)[P], T (&c)[P], T (&d)[P], int t) {
    T aL, cL, dL, aR, cR, dR;
    if constexpr (K < 5) {
        constexpr int AND = 0x1f & ~((2 << K) - 1);
        aL = swz<AND, (1 << K) - 1>(a[P - 1]);
        cL = swz<AND, (1 << K) - 1>(c[P - 1]);
        dL = swz<AND, (1 << K) - 1>(d[P - 1]);
        aR = swz<AND, (1 << K)>(a[0]);
        cR = swz<AND, (1 << K)>(c[0]);
        dR = swz<AND, (1 << K)>(d[0]);
    } else {
        aL = per_word(a[P - 1], [](int w) { return __builtin_amdgcn_readlane(w, 31); });
        cL = per_word(c[P - 1], [](int w) { return __builtin_amdgcn_readlane(w, 31); });
        dL = per_word(d[P - 1], [](int w) { return __builtin_amdgcn_readlane(w, 31); });
        aR = per_word(a[0], [](int w) { return __builtin_amdgcn_readlane(w, 32); });
        cR = per_word(c[0], [](int w) { return __builtin_amdgcn_readlane(w, 32); });
        dR = per_word(d[0], [](int w) { return __builtin_amdgcn_readlane(w, 32); });
    }
    const WmJoin<T> j = wm_join(aL, cL, dL, aR, cR, dR);
    const bool left = ((t >> K) & 1) == 0;
    const T al = left ? j.an : j.am, cl = left ? j.cn : j.cm, dl = left ? j.dn : j.dm;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const T u = left ? c[i] : a[i];  // the coefficient of the substituted unknown
        const T ka = left ? a[i] : T(0), kc = left ? T(0) : c[i];
        d[i] -= u * dl;
        a[i] = ka - u * al;
        c[i] = kc - u * cl;
    }
}

template <typename T, int P>
__device__ __forceinline__ void wave_wm(T (&a)[P], T (&c)[P], T (&d)[P], int t, int lps) {
    wm_inlane<T, P>(a, c, d);
    if (lps > 1) wm_lane_level<T, P, 0>(a, c, d, t);
    if (lps > 2) wm_lane_level<T, P, 1>(a, c, d, t);
    if (lps > 4) wm_lane_level<T, P, 2>(a, c, d, t);
    if (lps > 8) wm_lane_level<T, P, 3>(a, c, d, t);
    if (lps > 16) wm_lane_level<T, P, 4>(a, c, d, t);
    if (lps > 32) wm_lane_level<T, P, 5>(a, c, d, t);
}

// ---- Ladner-Fischer solver (PPX_TRI_LF)
//
// A block of consecutive equations is summarised by two equations, those of
// its first and of its last unknown, each in terms of the two unknowns just
// outside the block (the form of the Wang & Mou blocks above); two adjacent
// summaries combine with one join.  This combination is associative, so the
// summaries of the prefixes [0, i] follow from a scan with the
// Ladner-Fischer circuit; the last equation of prefix [0, i] reads
// x_i = d_i - c_i x_{i+1} (its a is 0: nothing lies before equation 0).  A
// second Ladner-Fischer scan, over the affine maps x_{i+1} -> x_i from the
// right, then gives every unknown.  In a lane:
//   1. the summary of its P equations, serially;
//   2. an inclusive scan of the lane summaries across the system's lanes
//      (at level K a lane of the upper half of each 2^(K+1)-lane block
//      combines the summary broadcast from the last lane of the lower half);
//   3. from the last equation of the previous lane's prefix, the forward
//      sweep over its own equations (one join each: the Thomas elimination);
//   4. the composition of its P maps, an inclusive scan of the lane maps
//      from the right (lower-half lanes take the upper half's first lane),
//      and the back substitution from the next lane's first unknown.

template <typename T>
struct TriEq {
    T a, c, d;
};

// Summary (f, l) of a block followed by (bf, bl) of the next: f takes the
// join's x_{m+1} term, l = bl its x_m term.
template <typename T>
__device__ __forceinline__ void lf_combine(TriEq<T> &f, TriEq<T> &l, const TriEq<T> &bf, const TriEq<T> &bl) {
    const WmJoin<T> j = wm_join(l.a, l.c, l.d, bf.a, bf.c, bf.d);
    wm_left(f.a, f.c, f.d, j);
    l = bl;
    wm_right(l.a, l.c, l.d, j);
}

template <int K, bool FROM_LOW, typename T>
__device__ __forceinline__ T lf_bcast(T v) {
    if constexpr (K < 5) {
        constexpr int AND = 0x1f & ~((2 << K) - 1);
        return swz<AND, FROM_LOW ? (1 << K) - 1 : (1 << K)>(v);
    } else {
        return per_word(v, [](int w) { return __builtin_amdgcn_readlane(w, FROM_LOW ? 31 : 32); });
    }
}

template <typename T, int K>
__device__ __forceinline__ void lf_prefix_level(TriEq<T> &f, TriEq<T> &l, int t) {
    TriEq<T> sf, sl;
    sf.a = lf_bcast<K, true>(f.a);
    sf.c = lf_bcast<K, true>(f.c);
    sf.d = lf_bcast<K, true>(f.d);
    sl.a = lf_bcast<K, true>(l.a);
    sl.c = lf_bcast<K, true>(l.c);
    sl.d = lf_bcast<K, true>(l.d);
    lf_combine(sf, sl, f, l);
    if ((t >> K) & 1) {
        f = sf;
        l = sl;
    }
}

template <typename T, int K>
__device__ __forceinline__ void lf_suffix_level(T &al, T &be, int t) {
    const T sa = lf_bcast<K, false>(al), sb = lf_bcast<K, false>(be);
    if (!((t >> K) & 1)) {  // own map after the upper half's: x = al - be * (sa - sb * Y)
        al -= be * sa;
        be = -(be * sb);
    }
}

template <typename T, int P>
__device__ __forceinline__ void wave_lf(T (&a)[P], T (&c)[P], T (&d)[P], int t, int lps) {
    // 1. the lane's summary
    TriEq<T> f{a[0], c[0], d[0]}, l = f;
#pragma unroll
    for (int j = 1; j < P; ++j) lf_combine(f, l, TriEq<T>{a[j], c[j], d[j]}, TriEq<T>{a[j], c[j], d[j]});
    // 2. prefix summaries of the lanes
    if (lps > 1) lf_prefix_level<T, 0>(f, l, t);
    if (lps > 2) lf_prefix_level<T, 1>(f, l, t);
    if (lps > 4) lf_prefix_level<T, 2>(f, l, t);
    if (lps > 8) lf_prefix_level<T, 3>(f, l, t);
    if (lps > 16) lf_prefix_level<T, 4>(f, l, t);
    if (lps > 32) lf_prefix_level<T, 5>(f, l, t);
    // 3. forward sweep from the previous lane's prefix (none for the first)
    T cq = sys_up(l.c, 1, lps), dq = sys_up(l.d, 1, lps);
    if (t == 0) cq = dq = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const T r = rcp(T(1) - cq * a[j]);
        dq = (d[j] - a[j] * dq) * r;
        cq = c[j] * r;
        c[j] = cq;
        d[j] = dq;
    }
    // 4. maps from the right and back substitution
    T al = d[P - 1], be = c[P - 1];
#pragma unroll
    for (int j = P - 2; j >= 0; --j) {
        al = d[j] - c[j] * al;
        be = -(c[j] * be);
    }
    if (lps > 1) lf_suffix_level<T, 0>(al, be, t);
    if (lps > 2) lf_suffix_level<T, 1>(al, be, t);
    if (lps > 4) lf_suffix_level<T, 2>(al, be, t);
    if (lps > 8) lf_suffix_level<T, 3>(al, be, t);
    if (lps > 16) lf_suffix_level<T, 4>(al, be, t);
    if (lps > 32) lf_suffix_level<T, 5>(al, be, t);
    T x = sys_down(al, 1, lps);  // first unknown of the next lane
    if (t == lps - 1) x = T(0);
#pragma unroll
    for (int j = P - 1; j >= 0; --j) {
        x = d[j] - c[j] * x;
        d[j] = x;
    }
}

// Boundary zeros, unit-diagonal scaling and the solve of the equations a
// lane holds (b is consumed; x ends in d).  tx: the thread's index in the
// workgroup (it selects the wave's LDS exchange buffer).
// Solutions of 64 bytes or more per lane leave through a per-wave LDS buffer
// (wave_store_staged): a non-temporal store of lane chunks that size covers
// only part of each line per instruction and measured slower than the
// default policy, while the staged form stores 64 consecutive 16-byte words
// per instruction.  Float64 PCR with 16 equations per lane keeps direct
// stores: staged, it measured 3-4% slower (alone and inside whole steps).
template <typename T, int ALGO, int P>
constexpr bool tri_staged_stores() {
    return P * (int)sizeof(T) >= 64 && !(ALGO == PPX_TRI_PCR_REG && sizeof(T) == 8 && P == 16);
}
// LDS values per wave of the in-wave kernels: the PCR_REG exchange buffer
// and the staging buffer share one region per wave.
template <typename T, int ALGO, int P>
constexpr int tri_wave_lds_vals() {
    constexpr int exch = ALGO == PPX_TRI_PCR_REG ? 3 * 64 * (P < 4 ? P : 4) : 0;
    constexpr int stage = tri_staged_stores<T, ALGO, P>() ? 64 * P : 0;
    return exch > stage ? exch : stage;
}

template <typename T, int ALGO, int P>
__device__ __forceinline__ void tridiag_wave_solve(T (&a)[P], const T (&b)[P], T (&c)[P], T (&d)[P], int t,
                                                   int lps, T *smem, int tx) {
    if (t == 0) a[0] = T(0);            // multiplies the absent x_{-1}
    if (t == lps - 1) c[P - 1] = T(0);  // multiplies the absent x_n
#pragma unroll
    for (int j = 0; j < P; ++j) {  // scale every row to unit diagonal
        const T r = rcp(b[j]);
        a[j] *= r;
        c[j] *= r;
        d[j] *= r;
    }
    if constexpr (ALGO == PPX_TRI_CR_SHFL) wave_cr<T, P>(a, c, d, t, lps);
    else if constexpr (ALGO == PPX_TRI_CR_PCR) wave_cr_pcr<T, P>(a, c, d, t, lps);
    else if constexpr (ALGO == PPX_TRI_PCR_SHFL) wave_pcr<T, P>(a, c, d, lps);
    else if constexpr (ALGO == PPX_TRI_WM) wave_wm<T, P>(a, c, d, t, lps);
    else if constexpr (ALGO == PPX_TRI_LF) wave_lf<T, P>(a, c, d, t, lps);
    else wave_pcr_reg<T, P>(a, c, d, t, lps, smem + (tx >> 6) * tri_wave_lds_vals<T, ALGO, P>());
}

// The solution of a wave whose lanes hold consecutive chunks of P values of
// one contiguous range (dst: the wave's first value; lanes at and beyond
// `active` store nothing): each lane writes its chunk to the wave's LDS
// buffer `buf` (64 P values), then lane l stores 16-byte words l, l + 64,
// ... of the range, non-temporal.  Words are XOR-swizzled within each lane's
// four (w ^ ((w >> 2) & 3)), which spreads a write instruction's lanes over
// the banks and leaves the reads, four consecutive words per group of four
// lanes, conflict-free.  A wave's LDS operations run in order; the fences
// only keep the compiler from moving them.
template <typename T, int P>
__device__ __forceinline__ void wave_store_staged(T *dst, const T (&v)[P], T *buf, int lane, int active) {
    constexpr int W = P * (int)sizeof(T) / 16;  // words per lane
    static_assert(W == 4 || W == 8, "staged stores are laid out for four or eight words per lane");
    constexpr int LW = W == 4 ? 2 : 3;
    u32x4 *bw = reinterpret_cast<u32x4 *>(buf);
    const auto phys = [](int w) { return w ^ ((w >> LW) & (W - 1)); };
#pragma unroll
    for (int j = 0; j < W; ++j) {
        u32x4 x;
        __builtin_memcpy(&x, &v[j * 16 / (int)sizeof(T)], 16);
        bw[phys(lane * W + j)] = x;
    }
    wave_lds_order();
    u32x4 *dw = reinterpret_cast<u32x4 *>(dst);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int w = lane + 64 * k;
        const u32x4 x = bw[phys(w)];
        if (w < active * W) store_nt(dw + w, x);
    }
    wave_lds_order();
}

// One workgroup's share: systems [first, first + nsys) of size n = P * lps,
// lps = n / P <= 64 lanes each; every lane owns P equations.  Lanes of
// systems beyond nsys solve identity rows and store nothing.  tx: the
// thread's index in the workgroup.
template <typename T, int ALGO, int P>
__device__ __forceinline__ void tridiag_wave_block(const T *A, const T *B, const T *C, const T *D,
                                                   T *X, int log2n, long long first, int nsys, T *smem, int tx) {
    const int n = 1 << log2n;
    const int lps = n / P;
    const int sys_local = tx / lps;
    const int t = tx % lps;
    const bool active = sys_local < nsys;
    const long long base = (first + sys_local) * n + (long long)t * P;
    T a[P], b[P], c[P], d[P];
    if (active) {
        wave_load<T, P>(A + base, a);
        wave_load<T, P>(B + base, b);
        wave_load<T, P>(C + base, c);
        wave_load<T, P>(D + base, d);
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            a[j] = c[j] = d[j] = T(0);
            b[j] = T(1);
        }
    }
    tridiag_wave_solve<T, ALGO, P>(a, b, c, d, t, lps, smem, tx);
    if constexpr (tri_staged_stores<T, ALGO, P>()) {
        // whole waves of consecutive threads: the wave's lanes cover the
        // contiguous range starting at its first thread's chunk
        if (blockDim.x % 64 == 0) {
            const int w0 = tx & ~63;
            const int active_lanes = max(0, min(64, nsys * lps - w0));
            wave_store_staged<T, P>(X + first * n + (long long)w0 * P, d,
                                    smem + (tx >> 6) * tri_wave_lds_vals<T, ALGO, P>(), tx & 63, active_lanes);
            return;
        }
    }
    if (active) wave_store<T, P>(X + base, d);
}

// ---- the CR -> PCR hybrid for systems spanning several waves
// (PPX_TRI_CR_PCR with 64 < n / P <= 1024)
//
// The same three phases as wave_cr_pcr, one system per n / P consecutive
// threads of the workgroup, but the lanes of a system cross waves, so every
// exchange between lanes goes through LDS slots indexed by the thread (xs:
// two sets of three arrays of L values, L = the workgroup's threads).  Each
// exchange writes one set, waits at a barrier and reads it; consecutive
// exchanges alternate sets, so a set is rewritten only after the barrier of
// the exchange in between, which every thread reaches after its reads of the
// set.  An absent neighbour (outside the system) is an identity row (zeros).
// Barriers: log2 P forward levels, log2(n / P) PCR steps, one for the
// previous lane's unknown.  Every thread of the workgroup reaches each of
// them (threads of absent systems solve identity rows).
template <typename T, int P>
__device__ __forceinline__ void block_cr_pcr(T (&a)[P], T (&c)[P], T (&d)[P], int t, int lps, int tx, int L,
                                             T *xs) {
    int set = 0;
    auto slots = [&]() {
        T *w = xs + (set & 1) * 3 * L;
        ++set;
        return w;
    };
    // ---- CR forward levels inside the lane
#pragma unroll
    for (int s = 1; 2 * s <= P; s *= 2) {
        T *w = slots();
        w[tx] = a[s - 1];
        w[L + tx] = c[s - 1];
        w[2 * L + tx] = d[s - 1];
        __syncthreads();
        T na = T(0), nc = T(0), nd = T(0);  // equation s - 1 of the next lane
        if (t + 1 < lps) {
            na = w[tx + 1];
            nc = w[L + tx + 1];
            nd = w[2 * L + tx + 1];
        }
#pragma unroll
        for (int r = 2 * s - 1; r < P; r += 2 * s) {
            const bool local = r + s < P;
            unit_eliminate(a[r], c[r], d[r], a[r - s], c[r - s], d[r - s], local ? a[(r + s) % P] : na,
                           local ? c[(r + s) % P] : nc, local ? d[(r + s) % P] : nd);
        }
    }
    // ---- PCR on the lanes' last equations
    for (int dl = 1; dl < lps; dl *= 2) {
        T *w = slots();
        w[tx] = a[P - 1];
        w[L + tx] = c[P - 1];
        w[2 * L + tx] = d[P - 1];
        __syncthreads();
        T la = T(0), lc = T(0), ld = T(0), ra = T(0), rc = T(0), rd = T(0);
        if (t >= dl) {
            la = w[tx - dl];
            lc = w[L + tx - dl];
            ld = w[2 * L + tx - dl];
        }
        if (t + dl < lps) {
            ra = w[tx + dl];
            rc = w[L + tx + dl];
            rd = w[2 * L + tx + dl];
        }
        unit_eliminate(a[P - 1], c[P - 1], d[P - 1], la, lc, ld, ra, rc, rd);
    }
    // ---- the previous lane's last unknown, then back substitution in the lane
    T *w = slots();
    w[tx] = d[P - 1];
    __syncthreads();
    const T xl = t > 0 ? w[tx - 1] : T(0);
#pragma unroll
    for (int s = P / 2; s >= 1; s /= 2) {
#pragma unroll
        for (int r = s - 1; r < P; r += 2 * s) {
            T x = d[r];
            if (r >= s) x -= a[r] * d[r - s];
            else x -= a[r] * xl;  // xl = 0 in the first lane, where a[0] = 0 too
            x -= c[r] * d[r + s];
            d[r] = x;
        }
    }
}

// One workgroup's share of the multi-wave hybrid: systems [first, first +
// nsys), lps = n / P > 64 lanes each (several waves), L = the workgroup's
// threads (a multiple of lps); xs holds 6 * L values.
template <typename T, int P>
__device__ __forceinline__ void tridiag_blk_block(const T *A, const T *B, const T *C, const T *D, T *X,
                                                  int log2n, long long first, int nsys, T *xs, int tx, int L) {
    const int n = 1 << log2n;
    const int lps = n / P;
    const int sys_local = tx / lps;
    const int t = tx % lps;
    const bool active = sys_local < nsys;
    const long long base = (first + sys_local) * n + (long long)t * P;
    T a[P], b[P], c[P], d[P];
    if (active) {
        wave_load<T, P>(A + base, a);
        wave_load<T, P>(B + base, b);
        wave_load<T, P>(C + base, c);
        wave_load<T, P>(D + base, d);
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            a[j] = c[j] = d[j] = T(0);
            b[j] = T(1);
        }
    }
    if (t == 0) a[0] = T(0);            // multiplies the absent x_{-1}
    if (t == lps - 1) c[P - 1] = T(0);  // multiplies the absent x_n
#pragma unroll
    for (int j = 0; j < P; ++j) {  // scale every row to unit diagonal
        const T r = rcp(b[j]);
        a[j] *= r;
        c[j] *= r;
        d[j] *= r;
    }
    block_cr_pcr<T, P>(a, c, d, t, lps, tx, L, xs);
    if (active) wave_store<T, P>(X + base, d);
}

template <typename T, int P>
__global__ __launch_bounds__(tri_blk_max_threads(sizeof(T), P)) void k_tridiag_blk(const T *a, const T *b, const T *c, const T *d, T *x,
                                                      int log2n, long long batch, int gb) {
    extern __shared__ float4 smem_raw[];  // 6 * blockDim.x values
    const long long first = (long long)blockIdx.x * gb;
    const int nsys = (int)min((long long)gb, batch - first);
    tridiag_blk_block<T, P>(a, b, c, d, x, log2n, first, nsys, reinterpret_cast<T *>(smem_raw), threadIdx.x,
                            blockDim.x);
}

// Minimum waves per SIMD the compiler must leave room for: 3 for 16 doubles
// per lane and array with CR or the LDS-exchange PCR (left alone it allocated
// up to 253 VGPRs there, two waves per SIMD, so the 16 systems per CU of an
// n = 1024 batch ran in two rounds), else no constraint (the shuffle PCR
// spills under it).
template <typename T, int ALGO, int P>
constexpr int tri_wave_min_waves() {
    return P * (int)sizeof(T) >= 128 && ALGO != PPX_TRI_PCR_SHFL ? 3 : 1;
}

template <typename T, int ALGO, int P>
__global__ __launch_bounds__(256, (tri_wave_min_waves<T, ALGO, P>())) void k_tridiag_wave(const T *a, const T *b, const T *c, const T *d,
                                                      T *x, int log2n, long long batch, int gb) {
    extern __shared__ float4 smem_raw[];  // PPX_TRI_PCR_REG: 3 * 64 * min(P, 4) values per wave
    const long long first = (long long)blockIdx.x * gb;
    const int nsys = (int)min((long long)gb, batch - first);
    tridiag_wave_block<T, ALGO, P>(a, b, c, d, x, log2n, first, nsys, reinterpret_cast<T *>(smem_raw), threadIdx.x);
}

// Persistent variant (algo | PPX_TRI_PIPE): a grid of resident workgroups
// (at most one per group) walks the groups of gb systems (g, g + gridDim.x,
// ...) and loads the next group's coefficients into a second register set
// while it solves the current one.  With every wave resident at once the
// plain kernel runs in one round, so all waves load, then all compute, then
// all store; here one group's loads overlap the previous group's solve.
// Loads and stores go through per-group buffer descriptors (lanes past the
// batch read zeros and store nothing, without a branch); the first iteration
// is peeled and the loop unrolled twice with the two register sets swapping
// roles, so the wait for the prefetched group never also covers the stores
// issued after it.  Lanes past the batch solve rows of zeros, whose
// non-finite results stay in their own lanes, as any system's do.
template <typename T, int ALGO, int P>
__global__ __launch_bounds__(256) void k_tridiag_wave_pipe(const T *A, const T *B, const T *C, const T *D,
                                                           T *X, int log2n, long long batch, int gb) {
    extern __shared__ float4 smem_raw[];
    T *smem = reinterpret_cast<T *>(smem_raw);
    const int n = 1 << log2n;
    const int lps = n / P;
    const int sys_local = threadIdx.x / lps;
    const int t = threadIdx.x % lps;
    const int voff = (sys_local * n + t * P) * (int)sizeof(T);  // byte offset within a group
    const long long ngroups = (batch + gb - 1) / gb;
    const long long G = gridDim.x;
    constexpr int es = sizeof(T);
    T a0[P], b0[P], c0[P], d0[P], a1[P], b1[P], c1[P], d1[P];
    auto load = [&](long long grp, T (&a)[P], T (&b)[P], T (&c)[P], T (&d)[P]) {
        buf_load<T, P>(a, group_rsrc(A, grp, gb, n, es, batch), voff);
        buf_load<T, P>(b, group_rsrc(B, grp, gb, n, es, batch), voff);
        buf_load<T, P>(c, group_rsrc(C, grp, gb, n, es, batch), voff);
        buf_load<T, P>(d, group_rsrc(D, grp, gb, n, es, batch), voff);
    };
    auto iteration = [&](long long grp, T (&a)[P], T (&b)[P], T (&c)[P], T (&d)[P], T (&na)[P], T (&nb)[P],
                         T (&nc)[P], T (&nd)[P]) {
        load(grp + G, na, nb, nc, nd);
        __builtin_amdgcn_sched_barrier(0);
        tridiag_wave_solve<T, ALGO, P>(a, b, c, d, t, lps, smem, threadIdx.x);
        buf_store<T, P, tri_nt_stores<T, P>() ? kStoreNT : 0>(d, group_rsrc(X, grp, gb, n, es, batch), voff);
    };
    long long g = blockIdx.x;  // < ngroups: the grid never exceeds the groups
    load(g, a0, b0, c0, d0);
    iteration(g, a0, b0, c0, d0, a1, b1, c1, d1);
    for (g += G; g < ngroups; g += 2 * G) {
        iteration(g, a1, b1, c1, d1, a0, b0, c0, d0);
        if (g + G >= ngroups) break;
        iteration(g + G, a0, b0, c0, d0, a1, b1, c1, d1);
    }
}

}  // namespace ppx
