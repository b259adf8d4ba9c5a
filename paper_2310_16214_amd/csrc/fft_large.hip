// Large-N batched FFT (2^14 < n <= 2^20) in two passes of column FFTs -- the
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
// A workgroup takes a tile of kTileCols = 16 adjacent columns: it reads them
// row by row (16 lanes on 16 consecutive values, 128-byte runs) into LDS,
// transforms the 16 columns with the single-pass stage code (radix R = P,
// T = len/P threads per column, exchanges in LDS), and writes the tile back
// the same way (pass B) or row by row (pass A, 512-byte runs per wave).  The
// LDS tile pads each column to len + 1 values, so that the 16 values a row
// read or write touches fall on different banks.
//
// The pass-A twiddles w_n^m (m < n <= 2^20) are the product of two table
// entries, w_{2^20}^{m' mod 1024} * w_{2^20}^{1024 (m' div 1024)} with
// m' = m * 2^20 / n: 2 x 1024 values built on the host in double precision.
#include "fft_device.h"

#include <map>
#include <mutex>

namespace ppx {

constexpr int kTileCols = 16;

__device__ __forceinline__ int tile_slot(int c, int e, int len) { return swz_c(c * (len + 1) + e); }

template <int R, int LOG2LEN, bool PASS_A>
__global__ __launch_bounds__(1024) void k_fft_tile(const float2 *in, float2 *out, const float2 *__restrict__ tw,
                                                    const float2 *__restrict__ tw_lo,
                                                    const float2 *__restrict__ tw_hi, int log2n,
                                                    int log2cols, long long tiles, float sgn) {
    constexpr int len = 1 << LOG2LEN;  // column length: the sub-transform size
    constexpr int P = R;
    constexpr int lT = LOG2LEN - clog2(P);
    constexpr int T = 1 << lT;
    extern __shared__ float4 lds_raw[];
    float2 *buf = reinterpret_cast<float2 *>(lds_raw);
    const long long prob = blockIdx.x / tiles;
    const int c0 = (int)(blockIdx.x % tiles) * kTileCols;
    const long long base = prob << log2n;
    const long long cols = 1LL << log2cols;
    for (int i = threadIdx.x; i < len * kTileCols; i += blockDim.x) {
        const int c = i & (kTileCols - 1), e = i >> 4;
        buf[tile_slot(c, e, len)] = in[base + e * cols + c0 + c];
    }
    __syncthreads();
    const int lp = threadIdx.x >> lT;  // column of the tile
    const int tid = threadIdx.x & (T - 1);
    float2 v[P];
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = buf[tile_slot(lp, tid + j * T, len)];
    __syncthreads();
    if constexpr (PASS_A) fft_conj<P>(v, sgn);  // the inverse: conjugated in pass A, out in pass B
    fft_stages_ct<R, P, false, LOG2LEN, 0, true>(v, buf, lp * (len + 1), nullptr, tid, true, sgn, tw);
    __syncthreads();
    if constexpr (PASS_A) {
        const int shift = 20 - log2n;
        for (int i = threadIdx.x; i < len * kTileCols; i += blockDim.x) {
            const int e = i & (len - 1), c = i >> LOG2LEN;
            const unsigned m = ((unsigned)(c0 + c) * (unsigned)e) << shift;  // < 2^20
            const float2 w = cmul(tw_lo[m & 1023u], tw_hi[m >> 10]);
            store_nt_any(out + base + (long long)(c0 + c) * len + e, cmul(buf[tile_slot(c, e, len)], w));
        }
    } else {
        for (int i = threadIdx.x; i < len * kTileCols; i += blockDim.x) {
            const int c = i & (kTileCols - 1), e = i >> 4;
            const float2 y = buf[tile_slot(c, e, len)];
            store_nt_any(out + base + e * cols + c0 + c, make_float2(y.x, sgn * y.y));
        }
    }
}

using TileKernel = void (*)(const float2 *, float2 *, const float2 *, const float2 *, const float2 *, int, int,
                            long long, float);

template <bool A>
static TileKernel tile_lookup(int radix, int log2len) {
    if (radix == 16) {
        switch (log2len) {
            case 6: return &k_fft_tile<16, 6, A>;
            case 7: return &k_fft_tile<16, 7, A>;
            case 8: return &k_fft_tile<16, 8, A>;
            case 9: return &k_fft_tile<16, 9, A>;
            case 10: return &k_fft_tile<16, 10, A>;
            default: return nullptr;
        }
    }
    if (radix == 8) {
        switch (log2len) {
            case 5: return &k_fft_tile<8, 5, A>;
            case 6: return &k_fft_tile<8, 6, A>;
            case 7: return &k_fft_tile<8, 7, A>;
            case 8: return &k_fft_tile<8, 8, A>;
            case 9: return &k_fft_tile<8, 9, A>;
            default: return nullptr;
        }
    }
    return nullptr;
}

const void *fft_tile_kernel(int radix, int log2len, bool pass_a) {
    return reinterpret_cast<const void *>(pass_a ? tile_lookup<true>(radix, log2len)
                                                 : tile_lookup<false>(radix, log2len));
}

bool fft_tile_shape_valid(int radix, int log2len) {
    if (radix != 8 && radix != 16) return false;
    const int threads = kTileCols * ((1 << log2len) / radix);
    return threads >= 64 && threads <= 1024 && tile_lookup<true>(radix, log2len) != nullptr;
}

int64_t fft_tile_lds_bytes(int log2len) {
    const int64_t vals = (int64_t)kTileCols * ((1 << log2len) + 1);
    return (vals + 255) / 256 * 256 * (int64_t)sizeof(float2);  // the swizzle stays in aligned 256-value blocks
}

void fft_large_host_twiddles(float *lo2, float *hi2) {
    const double two_pi = 6.283185307179586476925286766559;
    for (int j = 0; j < 1024; ++j) {
        const double a = two_pi * (double)j / (double)(1 << 20), b = two_pi * (double)j / 1024.0;
        lo2[2 * j] = (float)cos(a);
        lo2[2 * j + 1] = (float)(-sin(a));
        hi2[2 * j] = (float)cos(b);
        hi2[2 * j + 1] = (float)(-sin(b));
    }
}

// ---------------------------------------------------------------- plans

int fft_plan_check(int64_t n, const ppx_fft_plan &p) {
    if (!is_pow2(n) || n <= PPX_MAX_N || n > PPX_MAX_N_LARGE)
        return fail(PPX_EINVAL, "large FFT: n must be a power of two in (16384, 1048576]");
    const int ln = ilog2(n);
    if (p.log2_n1 < 1 || p.log2_n1 >= ln) return fail(PPX_ECONFIG, "plan: log2_n1 out of range");
    if (!fft_tile_shape_valid(p.radix_a, ln - p.log2_n1))
        return fail(PPX_ECONFIG, "plan: radix_a does not support column length n / n1");
    if (!fft_tile_shape_valid(p.radix_b, p.log2_n1))
        return fail(PPX_ECONFIG, "plan: radix_b does not support column length n1");
    return PPX_OK;
}

std::vector<ppx_fft_plan> fft_enumerate_plans(int64_t n) {
    std::vector<ppx_fft_plan> out;
    if (!is_pow2(n) || n <= PPX_MAX_N || n > PPX_MAX_N_LARGE) return out;
    const int ln = ilog2(n);
    for (int l1 = 1; l1 < ln; ++l1)
        for (int ra : {8, 16})
            for (int rb : {8, 16}) {
                const ppx_fft_plan p{l1, ra, rb};
                if (fft_tile_shape_valid(ra, ln - l1) && fft_tile_shape_valid(rb, l1)) out.push_back(p);
            }
    return out;
}

void fft_default_plan(int64_t n, ppx_fft_plan &p) {
    const int ln = ilog2(n);
    p = ppx_fft_plan{0, 0, 0};
    for (int l1 = ln / 2; l1 >= 1; --l1) {  // the most even split with n1 <= n2
        for (int ra : {8, 16})
            for (int rb : {8, 16})
                if (fft_tile_shape_valid(ra, ln - l1) && fft_tile_shape_valid(rb, l1) && !p.log2_n1)
                    p = ppx_fft_plan{l1, ra, rb};
        if (p.log2_n1) return;
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

int launch_fft_large(const void *in, void *out, int log2n, int64_t batch, const ppx_fft_plan &p, bool inverse,
                     hipStream_t s) {
    const DeviceInfo *di = device_info();
    if (!di) return PPX_EDEVICE;
    const int l1 = p.log2_n1, l2 = log2n - l1;
    TileKernel ka = tile_lookup<true>(p.radix_a, l2), kb = tile_lookup<false>(p.radix_b, l1);
    if (!ka || !kb) return fail(PPX_ECONFIG, "no tile kernel for this plan");
    const float sgn = inverse ? -1.0f : 1.0f;
    const float2 *tw = static_cast<const float2 *>(di->twiddles);
    const float2 *lo = static_cast<const float2 *>(di->twiddles_large_lo);
    const float2 *hi = static_cast<const float2 *>(di->twiddles_large_hi);
    // pass A: columns of length n2 of the [n2][n1] input, tiles of 16 of the n1 columns
    const long long tiles_a = (1LL << l1) / kTileCols, tiles_b = (1LL << l2) / kTileCols;
    hipLaunchKernelGGL(ka, dim3((unsigned)(batch * tiles_a)), dim3(kTileCols * ((1 << l2) / p.radix_a)),
                       (size_t)fft_tile_lds_bytes(l2), s, static_cast<const float2 *>(in), static_cast<float2 *>(out),
                       tw, lo, hi, log2n, l1, tiles_a, sgn);
    int rc = fail_hip(hipGetLastError(), "large FFT pass A launch");
    if (rc) return rc;
    // pass B: columns of length n1 of the [n1][n2] intermediate, in place
    hipLaunchKernelGGL(kb, dim3((unsigned)(batch * tiles_b)), dim3(kTileCols * ((1 << l1) / p.radix_b)),
                       (size_t)fft_tile_lds_bytes(l1), s, static_cast<const float2 *>(out), static_cast<float2 *>(out),
                       tw, lo, hi, log2n, l2, tiles_b, sgn);
    return fail_hip(hipGetLastError(), "large FFT pass B launch");
}

}  // namespace ppx
