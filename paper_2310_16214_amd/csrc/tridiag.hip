// Host launcher of the kernels in tridiag_device.h.
#include "tridiag_device.h"
#include "tridiag_wave_device.h"

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

namespace ppx {

// ------------------------------------------------------------------- host

int64_t tridiag_lds_bytes(int n, const ppx_config &c, int dtype) {
    const int64_t es = dtype == PPX_F64 ? 8 : 4;
    const int64_t P = c.elems_per_thread > 0 ? c.elems_per_thread
                                             : (int64_t)n * c.problems_per_block / c.threads_per_block;
    if (tri_blk(c.algo, n, P)) return 6 * (int64_t)c.threads_per_block * es;  // two sets of a, c, d slots
    if (tri_in_wave(c.algo)) {
        // per wave: the PCR_REG exchange buffer (3 * 64 * min(P, 4) values)
        // and the staging buffer of solution chunks of 64 bytes or more
        // (64 * P values) share one region (tri_wave_lds_vals,
        // tri_staged_stores)
        const int64_t waves = (c.threads_per_block + 63) / 64;
        const bool pcr_reg = tri_base(c.algo) == PPX_TRI_PCR_REG;
        const int64_t exch = pcr_reg ? 3 * 64 * (P < 4 ? P : 4) : 0;
        const int64_t stage = P * es >= 64 && !(pcr_reg && es == 8 && P == 16) ? 64 * P : 0;
        return waves * (exch > stage ? exch : stage) * es;
    }
    return tri_lds_arrays(c.algo) * es * (int64_t)c.problems_per_block * n;
}

template <typename T, int A, int P, bool PIPE>
static const void *wave_entry() {
    if constexpr (!PIPE) return reinterpret_cast<const void *>(&k_tridiag_wave<T, A, P>);
    else if constexpr (P * (int)sizeof(T) <= kTriPipeMaxBytes)
        return reinterpret_cast<const void *>(&k_tridiag_wave_pipe<T, A, P>);
    else return nullptr;
}

template <typename T, int A, bool PIPE>
static const void *wave_kernel_p(int P) {
    switch (P) {
        case 2: return wave_entry<T, A, 2, PIPE>();
        case 4: return wave_entry<T, A, 4, PIPE>();
        case 8: return wave_entry<T, A, 8, PIPE>();
        case 16: return wave_entry<T, A, 16, PIPE>();
        default: return nullptr;
    }
}

template <typename T, bool PIPE>
static const void *wave_kernel(int base, int P) {
    switch (base) {
        case PPX_TRI_CR_PCR: return wave_kernel_p<T, PPX_TRI_CR_PCR, PIPE>(P);
        case PPX_TRI_CR_SHFL: return wave_kernel_p<T, PPX_TRI_CR_SHFL, PIPE>(P);
        case PPX_TRI_PCR_SHFL: return wave_kernel_p<T, PPX_TRI_PCR_SHFL, PIPE>(P);
        case PPX_TRI_PCR_REG: return wave_kernel_p<T, PPX_TRI_PCR_REG, PIPE>(P);
        case PPX_TRI_WM: return wave_kernel_p<T, PPX_TRI_WM, PIPE>(P);
        case PPX_TRI_LF: return wave_kernel_p<T, PPX_TRI_LF, PIPE>(P);
        default: return nullptr;
    }
}

template <typename T>
using TriKernel = void (*)(const T *, const T *, const T *, const T *, T *, int, long long, int);

template <typename T>
static const void *blk_kernel(int P) {
    switch (P) {
        case 2: return reinterpret_cast<const void *>(&k_tridiag_blk<T, 2>);
        case 4: return reinterpret_cast<const void *>(&k_tridiag_blk<T, 4>);
        case 8: return reinterpret_cast<const void *>(&k_tridiag_blk<T, 8>);
        case 16: return reinterpret_cast<const void *>(&k_tridiag_blk<T, 16>);
        default: return nullptr;
    }
}

const void *tridiag_kernel(int dtype, int algo, int P, int64_t n) {
    const int base = tri_base(algo);
    const bool pipe = (algo & PPX_TRI_PIPE) != 0;
    if (tri_blk(algo, n, P)) {
        if (pipe) return nullptr;
        return dtype == PPX_F64 ? blk_kernel<double>(P) : dtype == PPX_F32 ? blk_kernel<float>(P) : nullptr;
    }
    if (tri_in_wave(algo)) {
        if (dtype == PPX_F64) return pipe ? wave_kernel<double, true>(base, P) : wave_kernel<double, false>(base, P);
        if (dtype == PPX_F32) return pipe ? wave_kernel<float, true>(base, P) : wave_kernel<float, false>(base, P);
        return nullptr;
    }
    if (pipe) return nullptr;
    if (dtype == PPX_F32) {
        if (algo == PPX_TRI_CR) return reinterpret_cast<const void *>(&k_tridiag<float, PPX_TRI_CR>);
        if (algo == PPX_TRI_PCR) return reinterpret_cast<const void *>(&k_tridiag<float, PPX_TRI_PCR>);
    } else if (dtype == PPX_F64) {
        if (algo == PPX_TRI_CR) return reinterpret_cast<const void *>(&k_tridiag<double, PPX_TRI_CR>);
        if (algo == PPX_TRI_PCR) return reinterpret_cast<const void *>(&k_tridiag<double, PPX_TRI_PCR>);
    }
    return nullptr;
}

// Resident workgroups per CU of a persistent kernel at (L, LDS bytes), from
// the occupancy query, made once per (kernel, L, LDS).
static int tri_resident_per_cu(const void *k, int L, int64_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, int64_t>, int> memo;
    const auto key = std::make_tuple(k, L, lds);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, L, (size_t)lds) != hipSuccess || nb < 1) nb = 1;
    std::lock_guard<std::mutex> lk(mu);
    memo[key] = nb;
    return nb;
}

template <typename T>
static int launch_t(const void *k, const void *a, const void *b, const void *c, const void *d,
                    void *x, int log2n, int64_t batch, const ppx_config &cfg, size_t lds,
                    int64_t grid, hipStream_t s) {
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
    const void *k = tridiag_kernel(dtype, cfg.algo, cfg.elems_per_thread, int64_t(1) << log2n);
    if (!k) return fail(PPX_ECONFIG, "no tridiagonal kernel for this dtype / algo");
    const int64_t lds = tridiag_lds_bytes(1 << log2n, cfg, dtype);
    if (lds > di->lds_per_block)
        return fail(PPX_ECONFIG, "tridiagonal configuration exceeds the LDS per workgroup");
    int64_t grid = (batch + cfg.problems_per_block - 1) / cfg.problems_per_block;
    if (cfg.algo & PPX_TRI_PIPE) {  // persistent: at most the resident workgroups
        const int64_t resident = (int64_t)tri_resident_per_cu(k, cfg.threads_per_block, lds) * di->cus;
        if (resident < grid) grid = resident;
    }
    if (dtype == PPX_F64) return launch_t<double>(k, a, b, c, d, x, log2n, batch, cfg, (size_t)lds, grid, s);
    return launch_t<float>(k, a, b, c, d, x, log2n, batch, cfg, (size_t)lds, grid, s);
}

}  // namespace ppx
