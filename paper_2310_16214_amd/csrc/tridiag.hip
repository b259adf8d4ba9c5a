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

template <typename T, int ALGO>
__global__ __launch_bounds__(1024) void k_tridiag(const T *a, const T *b, const T *c, const T *d,
                                                  T *x, int log2n, long long batch, int gb) {
    extern __shared__ float4 smem_raw[];
    T *smem = reinterpret_cast<T *>(smem_raw);
    const int n = 1 << log2n;
    const long long first = (long long)blockIdx.x * gb;
    const int nsys = (int)min((long long)gb, batch - first);
    const int total = nsys * n;
    const long long base = first * n;
    const int cap = gb * n;
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

// ------------------------------------------------------------------- host

int64_t tridiag_lds_bytes(int n, int gb, int dtype, int algo) {
    const int64_t es = dtype == PPX_F64 ? 8 : 4;
    return (algo == PPX_TRI_PCR ? 8 : 4) * es * (int64_t)gb * n;
}

template <typename T>
using TriKernel = void (*)(const T *, const T *, const T *, const T *, T *, int, long long, int);

const void *tridiag_kernel(int dtype, int algo) {
    if (dtype == PPX_F32) {
        if (algo == PPX_TRI_CR) return reinterpret_cast<const void *>(&k_tridiag<float, PPX_TRI_CR>);
        if (algo == PPX_TRI_PCR) return reinterpret_cast<const void *>(&k_tridiag<float, PPX_TRI_PCR>);
    } else if (dtype == PPX_F64) {
        if (algo == PPX_TRI_CR) return reinterpret_cast<const void *>(&k_tridiag<double, PPX_TRI_CR>);
        if (algo == PPX_TRI_PCR) return reinterpret_cast<const void *>(&k_tridiag<double, PPX_TRI_PCR>);
    }
    return nullptr;
}

template <typename T>
static int launch_t(const void *k, const void *a, const void *b, const void *c, const void *d,
                    void *x, int log2n, int64_t batch, const ppx_config &cfg, size_t lds,
                    hipStream_t s) {
    const int64_t grid = (batch + cfg.problems_per_block - 1) / cfg.problems_per_block;
    hipLaunchKernelGGL(reinterpret_cast<TriKernel<T>>(const_cast<void *>(k)), dim3((unsigned)grid),
                       dim3(cfg.threads_per_block), lds, s, static_cast<const T *>(a),
                       static_cast<const T *>(b), static_cast<const T *>(c),
                       static_cast<const T *>(d), static_cast<T *>(x), log2n, (long long)batch,
                       cfg.problems_per_block);
    return fail_hip(hipGetLastError(), "tridiag launch");
}

int launch_tridiag(const void *a, const void *b, const void *c, const void *d, void *x, int log2n,
                   int64_t batch, int dtype, const ppx_config &cfg, hipStream_t s) {
    const DeviceInfo *di = device_info();
    if (!di) return PPX_EDEVICE;
    const void *k = tridiag_kernel(dtype, cfg.algo);
    if (!k) return fail(PPX_ECONFIG, "no tridiagonal kernel for this dtype / algo");
    const int64_t lds = tridiag_lds_bytes(1 << log2n, cfg.problems_per_block, dtype, cfg.algo);
    if (lds > di->lds_per_block)
        return fail(PPX_ECONFIG, "tridiagonal configuration exceeds the LDS per workgroup");
    if (dtype == PPX_F64) return launch_t<double>(k, a, b, c, d, x, log2n, batch, cfg, (size_t)lds, s);
    return launch_t<float>(k, a, b, c, d, x, log2n, batch, cfg, (size_t)lds, s);
}

}  // namespace ppx
