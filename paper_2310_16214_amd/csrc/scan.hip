// Host launcher of the kernels in scan_device.h.
#include "scan_device.h"

#include <map>
#include <mutex>
#include <tuple>

namespace ppx {

// ------------------------------------------------------------------- host

int64_t scan_lds_bytes(int, int, int, int) { return 0; }

template <typename T>
using ScanKernel = void (*)(const T *, T *, int, long long, int);

template <typename T, int A, bool PIPE, bool EXCL>
static const void *scan_lookup_t(int P) {
#define PPX_SCAN_CASE(PV)                                                                  \
    case PV:                                                                               \
        return PIPE ? (const void *)&k_scan_pipe<T, PV, A, EXCL> : (const void *)&k_scan<T, PV, A, EXCL>;
    switch (P) {
        PPX_SCAN_CASE(2)
        PPX_SCAN_CASE(4)
        PPX_SCAN_CASE(8)
        PPX_SCAN_CASE(16)
        default:
            break;
    }
    // 32 values of 8 bytes (and a second set in the persistent variant) do
    // not fit the registers of a 1024-thread workgroup: float64 stops at 16.
    if constexpr (sizeof(T) == 4) {
        switch (P) {
            PPX_SCAN_CASE(32)
            default:
                break;
        }
    }
#undef PPX_SCAN_CASE
    return nullptr;
}

template <typename T, bool EXCL>
static const void *scan_lookup_a(int P, int algo) {
    switch (algo) {
        case PPX_SCAN_KS: return scan_lookup_t<T, PPX_SCAN_KS, false, EXCL>(P);
        case PPX_SCAN_LF: return scan_lookup_t<T, PPX_SCAN_LF, false, EXCL>(P);
        case PPX_SCAN_KS_PIPE: return scan_lookup_t<T, PPX_SCAN_KS, true, EXCL>(P);
        case PPX_SCAN_LF_PIPE: return scan_lookup_t<T, PPX_SCAN_LF, true, EXCL>(P);
        default: return nullptr;
    }
}

template <bool EXCL>
static const void *scan_kernel_x(int dtype, int P, int algo) {
    if (dtype == PPX_I32) return scan_lookup_a<int, EXCL>(P, algo);
    if (dtype == PPX_F32) return scan_lookup_a<float, EXCL>(P, algo);
    if (dtype == PPX_F64) return scan_lookup_a<double, EXCL>(P, algo);
    return nullptr;
}

const void *scan_kernel(int dtype, int P, int algo, bool exclusive) {
    return exclusive ? scan_kernel_x<true>(dtype, P, algo) : scan_kernel_x<false>(dtype, P, algo);
}

// Resident workgroups per CU of a persistent kernel at L threads, from the
// occupancy query, made once per (kernel, L).
static int scan_resident_per_cu(const void *k, int L) {
    static std::mutex mu;
    static std::map<std::tuple<const void *, int>, int> memo;
    const auto key = std::make_tuple(k, L);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, L, 0) != hipSuccess || nb < 1) nb = 1;
    std::lock_guard<std::mutex> lk(mu);
    memo[key] = nb;
    return nb;
}

template <typename T>
static void launch_t(const void *k, dim3 g, dim3 b, hipStream_t s, const void *in, void *out,
                     int log2n, int64_t batch, int gb) {
    hipLaunchKernelGGL(reinterpret_cast<ScanKernel<T>>(const_cast<void *>(k)), g, b, 0, s,
                       static_cast<const T *>(in), static_cast<T *>(out), log2n, (long long)batch, gb);
}

int launch_scan(const void *in, void *out, int log2n, int64_t batch, int dtype, const ppx_config &c,
                hipStream_t s, bool exclusive) {
    const void *k = scan_kernel(dtype, c.elems_per_thread, c.algo, exclusive);
    if (!k) return fail(PPX_ECONFIG, "no scan kernel for this dtype / elements-per-thread / algo");
    int64_t grid = (batch + c.problems_per_block - 1) / c.problems_per_block;
    if (c.algo & PPX_SCAN_KS_PIPE) {  // persistent: at most the resident workgroups
        const DeviceInfo *di = device_info();
        if (!di) return PPX_EDEVICE;
        const int64_t resident = (int64_t)scan_resident_per_cu(k, c.threads_per_block) * di->cus;
        if (resident < grid) grid = resident;
    }
    const dim3 g((unsigned)grid), b(c.threads_per_block);
    if (dtype == PPX_I32) launch_t<int>(k, g, b, s, in, out, log2n, batch, c.problems_per_block);
    else if (dtype == PPX_F32) launch_t<float>(k, g, b, s, in, out, log2n, batch, c.problems_per_block);
    else launch_t<double>(k, g, b, s, in, out, log2n, batch, c.problems_per_block);
    return fail_hip(hipGetLastError(), "scan launch");
}

}  // namespace ppx
