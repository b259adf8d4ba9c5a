// Host launcher of the kernels in scan_device.h.
#include "scan_device.h"

namespace ppx {

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
