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

template <typename T, int A, bool PIPE>
static const void *scan_lookup_t(int P) {
    switch (P) {
        case 2: return PIPE ? (const void *)&k_scan_pipe<T, 2, A> : (const void *)&k_scan<T, 2, A>;
        case 4: return PIPE ? (const void *)&k_scan_pipe<T, 4, A> : (const void *)&k_scan<T, 4, A>;
        case 8: return PIPE ? (const void *)&k_scan_pipe<T, 8, A> : (const void *)&k_scan<T, 8, A>;
        case 16: return PIPE ? (const void *)&k_scan_pipe<T, 16, A> : (const void *)&k_scan<T, 16, A>;
        case 32: return PIPE ? (const void *)&k_scan_pipe<T, 32, A> : (const void *)&k_scan<T, 32, A>;
        default: return nullptr;
    }
}

template <typename T>
static const void *scan_lookup_a(int P, int algo) {
    switch (algo) {
        case PPX_SCAN_KS: return scan_lookup_t<T, PPX_SCAN_KS, false>(P);
        case PPX_SCAN_LF: return scan_lookup_t<T, PPX_SCAN_LF, false>(P);
        case PPX_SCAN_KS_PIPE: return scan_lookup_t<T, PPX_SCAN_KS, true>(P);
        case PPX_SCAN_LF_PIPE: return scan_lookup_t<T, PPX_SCAN_LF, true>(P);
        default: return nullptr;
    }
}

const void *scan_kernel(int dtype, int P, int algo) {
    if (dtype == PPX_I32) return scan_lookup_a<int>(P, algo);
    if (dtype == PPX_F32) return scan_lookup_a<float>(P, algo);
    return nullptr;
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

int launch_scan(const void *in, void *out, int log2n, int64_t batch, int dtype, const ppx_config &c,
                hipStream_t s) {
    const void *k = scan_kernel(dtype, c.elems_per_thread, c.algo);
    if (!k) return fail(PPX_ECONFIG, "no scan kernel for this dtype / elements-per-thread / algo");
    int64_t grid = (batch + c.problems_per_block - 1) / c.problems_per_block;
    if (c.algo & PPX_SCAN_KS_PIPE) {  // persistent: at most the resident workgroups
        const DeviceInfo *di = device_info();
        if (!di) return PPX_EDEVICE;
        const int64_t resident = (int64_t)scan_resident_per_cu(k, c.threads_per_block) * di->cus;
        if (resident < grid) grid = resident;
    }
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
