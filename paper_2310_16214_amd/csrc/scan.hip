// Batched inclusive sum scan (Sec. III "Scan Operator" of arXiv:2310.16214),
// int32 (modulo 2^32) and float32, for gfx950.
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
//   4. add the exclusive prefix to the P values and store.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"
#include "ppx_internal.h"

namespace ppx {

template <typename T, int P>
__device__ __forceinline__ void load_chunk(const T *src, T (&v)[P]) {
    if constexpr (P * sizeof(T) % 16 == 0) {
        const int4 *s4 = reinterpret_cast<const int4 *>(src);
#pragma unroll
        for (int j = 0; j < (int)(P * sizeof(T) / 16); ++j) {
            const int4 w = s4[j];
            v[4 * j + 0] = __builtin_bit_cast(T, w.x);
            v[4 * j + 1] = __builtin_bit_cast(T, w.y);
            v[4 * j + 2] = __builtin_bit_cast(T, w.z);
            v[4 * j + 3] = __builtin_bit_cast(T, w.w);
        }
    } else {
        const int2 *s2 = reinterpret_cast<const int2 *>(src);
#pragma unroll
        for (int j = 0; j < P / 2; ++j) {
            const int2 w = s2[j];
            v[2 * j + 0] = __builtin_bit_cast(T, w.x);
            v[2 * j + 1] = __builtin_bit_cast(T, w.y);
        }
    }
}

template <typename T, int P>
__device__ __forceinline__ void store_chunk(T *dst, const T (&v)[P]) {
    if constexpr (P * sizeof(T) % 16 == 0) {
        int4 *d4 = reinterpret_cast<int4 *>(dst);
#pragma unroll
        for (int j = 0; j < (int)(P * sizeof(T) / 16); ++j)
            d4[j] = make_int4(__builtin_bit_cast(int, v[4 * j]), __builtin_bit_cast(int, v[4 * j + 1]),
                              __builtin_bit_cast(int, v[4 * j + 2]), __builtin_bit_cast(int, v[4 * j + 3]));
    } else {
        int2 *d2 = reinterpret_cast<int2 *>(dst);
#pragma unroll
        for (int j = 0; j < P / 2; ++j)
            d2[j] = make_int2(__builtin_bit_cast(int, v[2 * j]), __builtin_bit_cast(int, v[2 * j + 1]));
    }
}

template <typename T, int P, int ALGO>
__global__ __launch_bounds__(1024) void k_scan(const T *in, T *out, int log2n, long long batch,
                                               int gb) {
    __shared__ T wave_tot[kMaxThreadsPerBlock / kWave];
    constexpr int LP = P == 2 ? 1 : P == 4 ? 2 : P == 8 ? 3 : P == 16 ? 4 : 5;
    // integer adds wrap modulo 2^32: do them on unsigned values
    using U = typename std::conditional<std::is_same<T, int>::value, unsigned, T>::type;
    const int lT = log2n - LP;  // log2 threads per problem
    const int lp = threadIdx.x >> lT;
    const long long prob = (long long)blockIdx.x * gb + lp;
    const bool active = prob < batch;
    const long long off = (long long)blockIdx.x * gb * (1LL << log2n) + (long long)threadIdx.x * P;

    U v[P];
    if (active) {
        load_chunk<U, P>(reinterpret_cast<const U *>(in) + off, v);
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] = U(0);
    }
    // 1. serial scan within the thread
#pragma unroll
    for (int j = 1; j < P; ++j) v[j] = v[j] + v[j - 1];
    const U total = v[P - 1];

    // 2. lane network over the problem's segment of the wave
    const int lane = threadIdx.x & (kWave - 1);
    const int seg = lT >= 6 ? kWave : (1 << lT);
    U incl = ALGO == PPX_SCAN_LF ? lanes_scan_lf<U>(total, seg, lane)
                                 : lanes_scan_ks<U>(total, seg, lane);
    U prefix = incl - total;  // exclusive prefix of this thread within the wave segment

    // 3. earlier waves of the same problem
    if (lT > 6) {
        const int w = threadIdx.x >> 6;
        if (lane == kWave - 1) wave_tot[w] = __builtin_bit_cast(T, incl);
        __syncthreads();
        const int w0 = w & ~((1 << (lT - 6)) - 1);
        for (int u = w0; u < w; ++u) prefix = prefix + __builtin_bit_cast(U, wave_tot[u]);
    }

    // 4. add the prefix and store
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = v[j] + prefix;
    if (active) store_chunk<U, P>(reinterpret_cast<U *>(out) + off, v);
}

// ------------------------------------------------------------------- host

int64_t scan_lds_bytes(int, int, int, int) { return 0; }

template <typename T>
using ScanKernel = void (*)(const T *, T *, int, long long, int);

template <typename T, int A>
static const void *scan_lookup_t(int P) {
    switch (P) {
        case 2: return reinterpret_cast<const void *>(&k_scan<T, 2, A>);
        case 4: return reinterpret_cast<const void *>(&k_scan<T, 4, A>);
        case 8: return reinterpret_cast<const void *>(&k_scan<T, 8, A>);
        case 16: return reinterpret_cast<const void *>(&k_scan<T, 16, A>);
        case 32: return reinterpret_cast<const void *>(&k_scan<T, 32, A>);
        default: return nullptr;
    }
}

const void *scan_kernel(int dtype, int P, int algo) {
    if (algo != PPX_SCAN_KS && algo != PPX_SCAN_LF) return nullptr;
    if (dtype == PPX_I32)
        return algo == PPX_SCAN_LF ? scan_lookup_t<int, PPX_SCAN_LF>(P) : scan_lookup_t<int, PPX_SCAN_KS>(P);
    if (dtype == PPX_F32)
        return algo == PPX_SCAN_LF ? scan_lookup_t<float, PPX_SCAN_LF>(P) : scan_lookup_t<float, PPX_SCAN_KS>(P);
    return nullptr;
}

int launch_scan(const void *in, void *out, int log2n, int64_t batch, int dtype, const ppx_config &c,
                hipStream_t s) {
    const void *k = scan_kernel(dtype, c.elems_per_thread, c.algo);
    if (!k) return fail(PPX_ECONFIG, "no scan kernel for this dtype / elements-per-thread / algo");
    const int64_t grid = (batch + c.problems_per_block - 1) / c.problems_per_block;
    const dim3 g((unsigned)grid), b(c.threads_per_block);
    if (dtype == PPX_I32) {
        hipLaunchKernelGGL(reinterpret_cast<ScanKernel<int>>(const_cast<void *>(k)), g, b, 0, s,
                           static_cast<const int *>(in), static_cast<int *>(out), log2n,
                           (long long)batch, c.problems_per_block);
    } else {
        hipLaunchKernelGGL(reinterpret_cast<ScanKernel<float>>(const_cast<void *>(k)), g, b, 0, s,
                           static_cast<const float *>(in), static_cast<float *>(out), log2n,
                           (long long)batch, c.problems_per_block);
    }
    return fail_hip(hipGetLastError(), "scan launch");
}

}  // namespace ppx
