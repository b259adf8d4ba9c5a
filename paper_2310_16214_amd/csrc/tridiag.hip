// Host launcher of the kernels in tridiag_device.h.
#include "tridiag_device.h"
#include "tridiag_wave_device.h"

#include <type_traits>

namespace ppx {

// ------------------------------------------------------------------- host

int64_t tridiag_lds_bytes(int n, const ppx_config &c, int dtype) {
    const int64_t es = dtype == PPX_F64 ? 8 : 4;
    if (c.algo == PPX_TRI_PCR_REG) {  // exchange buffer: 3 * 64 * min(P, 4) values per wave
        const int64_t waves = (c.threads_per_block + 63) / 64;
        const int64_t P = c.elems_per_thread > 0 ? c.elems_per_thread
                                                 : (int64_t)n * c.problems_per_block / c.threads_per_block;
        return waves * 3 * 64 * (P < 4 ? P : 4) * es;
    }
    if (tri_in_wave(c.algo)) return 0;
    return tri_lds_arrays(c.algo) * es * (int64_t)c.problems_per_block * n;
}

template <typename T, int A>
static const void *wave_kernel_p(int P) {
    switch (P) {
        case 2: return reinterpret_cast<const void *>(&k_tridiag_wave<T, A, 2>);
        case 4: return reinterpret_cast<const void *>(&k_tridiag_wave<T, A, 4>);
        case 8: return reinterpret_cast<const void *>(&k_tridiag_wave<T, A, 8>);
        case 16: return reinterpret_cast<const void *>(&k_tridiag_wave<T, A, 16>);
        default: return nullptr;
    }
}

template <typename T>
using TriKernel = void (*)(const T *, const T *, const T *, const T *, T *, int, long long, int);

const void *tridiag_kernel(int dtype, int algo, int P) {
    if (algo == PPX_TRI_CR_SHFL)
        return dtype == PPX_F64 ? wave_kernel_p<double, PPX_TRI_CR_SHFL>(P) : dtype == PPX_F32 ? wave_kernel_p<float, PPX_TRI_CR_SHFL>(P) : nullptr;
    if (algo == PPX_TRI_PCR_SHFL)
        return dtype == PPX_F64 ? wave_kernel_p<double, PPX_TRI_PCR_SHFL>(P) : dtype == PPX_F32 ? wave_kernel_p<float, PPX_TRI_PCR_SHFL>(P) : nullptr;
    if (algo == PPX_TRI_PCR_REG)
        return dtype == PPX_F64 ? wave_kernel_p<double, PPX_TRI_PCR_REG>(P) : dtype == PPX_F32 ? wave_kernel_p<float, PPX_TRI_PCR_REG>(P) : nullptr;
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
    const void *k = tridiag_kernel(dtype, cfg.algo, cfg.elems_per_thread);
    if (!k) return fail(PPX_ECONFIG, "no tridiagonal kernel for this dtype / algo");
    const int64_t lds = tridiag_lds_bytes(1 << log2n, cfg, dtype);
    if (lds > di->lds_per_block)
        return fail(PPX_ECONFIG, "tridiagonal configuration exceeds the LDS per workgroup");
    if (dtype == PPX_F64) return launch_t<double>(k, a, b, c, d, x, log2n, batch, cfg, (size_t)lds, s);
    return launch_t<float>(k, a, b, c, d, x, log2n, batch, cfg, (size_t)lds, s);
}

}  // namespace ppx
