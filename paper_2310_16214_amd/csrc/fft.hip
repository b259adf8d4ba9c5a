// Host launcher of the kernels in fft_device.h.
#include "fft_device.h"

#include <map>
#include <mutex>
#include <tuple>

namespace ppx {

// ------------------------------------------------------------------- host

void fft_host_twiddles(float *out2) {
    const double two_pi = 6.283185307179586476925286766559;
    for (int m = 0; m < kNMax; ++m) {
        const double ang = two_pi * (double)m / (double)kNMax;
        out2[2 * m] = (float)cos(ang);
        out2[2 * m + 1] = (float)(-sin(ang));
    }
}

// The persistent kernels keep every stage's twiddle bases in LDS after the
// exchange buffer: per twiddled stage with span Ns, Ns entries of each of w^k,
// w^{4k}, w^{8k} that the radix reads (see k_fft_np).
static int64_t fft_pipe_twiddle_bytes(int n, int radix) {
    const int log2n = ilog2(n), lr = ilog2(radix);
    const int stages = (log2n + lr - 1) / lr - 1;
    const int per_k = 1 + (radix >= 8) + (radix >= 16);
    const int first = log2n % lr ? log2n % lr : lr;
    int64_t entries = 0;
    for (int i = 0; i < stages; ++i) entries += (int64_t)per_k << (first + i * lr);
    return entries * 8;
}

int64_t fft_lds_bytes(int n, int gb, int algo, int radix) {
    if (n <= radix) return 0;  // a single stage: no exchange
    const int64_t exch = (int64_t)gb * n * ((algo & PPX_FFT_LDS_SPLIT) ? 4 : 8);
    return exch + ((algo & PPX_FFT_LDS_PIPE) ? fft_pipe_twiddle_bytes(n, radix) : 0);
}

using FftKernel = void (*)(const float2 *, float2 *, const float2 *, int, long long, int, float);

template <int R, int P, bool S>
constexpr FftKernel fft_entry() {
    if constexpr (P >= R && P <= 32) return &k_fft<R, P, S>;
    else return nullptr;
}

template <int R, bool S>
constexpr FftKernel fft_entry_p(int lp) {
    return lp == 1 ? fft_entry<R, 2, S>() : lp == 2 ? fft_entry<R, 4, S>()
         : lp == 3 ? fft_entry<R, 8, S>() : lp == 4 ? fft_entry<R, 16, S>()
         : lp == 5 ? fft_entry<R, 32, S>() : nullptr;
}

template <bool S>
static FftKernel fft_lookup_s(int radix, int P) {
    const int lp = is_pow2(P) ? ilog2(P) : 0;
    switch (radix) {
        case 2: return fft_entry_p<2, S>(lp);
        case 4: return fft_entry_p<4, S>(lp);
        case 8: return fft_entry_p<8, S>(lp);
        case 16: return fft_entry_p<16, S>(lp);
        default: return nullptr;
    }
}

// The kernel of a configuration: the one specialised on log2 n where radix =
// P = 8 or 16 (the persistent variants exist only there) or radix = P = 4 and
// n <= 64, else the generic.  (The entry points take 16-byte aligned buffers
// only, which the specialised kernels' 16-byte staged accesses rely on.)
static FftKernel fft_lookup(int radix, int P, int algo, int log2n) {
    const bool split = (algo & PPX_FFT_LDS_SPLIT) != 0, pipe = (algo & PPX_FFT_LDS_PIPE) != 0;
    if (fft_pipe_available(radix, P)) {
        const void *k = P == 8 ? fft_spec8_kernel(log2n, split, pipe) : fft_spec16_kernel(log2n, split, pipe);
        if (k || pipe) return reinterpret_cast<FftKernel>(const_cast<void *>(k));
    }
    if (pipe) return nullptr;
    if (radix == 4 && P == 4) {
        if (const void *k = fft_spec4_kernel(log2n, split)) return reinterpret_cast<FftKernel>(const_cast<void *>(k));
    }
    return split ? fft_lookup_s<true>(radix, P) : fft_lookup_s<false>(radix, P);
}

const void *fft_kernel(int radix, int P, int algo, int log2n) {
    return reinterpret_cast<const void *>(fft_lookup(radix, P, algo, log2n));
}

// Resident workgroups per CU of a persistent kernel at (L, LDS bytes), from
// the occupancy query, made once per (kernel, L, LDS).
static int resident_blocks_per_cu(FftKernel k, int L, int64_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, int64_t>, int> memo;
    const auto key = std::make_tuple(reinterpret_cast<const void *>(k), L, lds);
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

int launch_fft(const void *in, void *out, int log2n, int64_t batch, const ppx_config &c,
               bool inverse, hipStream_t s) {
    const DeviceInfo *di = device_info();
    if (!di) return PPX_EDEVICE;
    FftKernel k = fft_lookup(c.radix, c.elems_per_thread, c.algo, log2n);
    if (!k) return fail(PPX_ECONFIG, "no FFT kernel for this radix / elements-per-thread");
    const int n = 1 << log2n;
    const int64_t lds = fft_lds_bytes(n, c.problems_per_block, c.algo, c.radix);
    if (lds > di->lds_per_block) return fail(PPX_ECONFIG, "FFT configuration exceeds the LDS per workgroup");
    int64_t grid = (batch + c.problems_per_block - 1) / c.problems_per_block;
    if (c.algo & PPX_FFT_LDS_PIPE) {  // persistent: at most the resident workgroups
        const int64_t resident = (int64_t)resident_blocks_per_cu(k, c.threads_per_block, lds) * di->cus;
        if (resident < grid) grid = resident;
    }
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(c.threads_per_block), (size_t)lds, s,
                       static_cast<const float2 *>(in), static_cast<float2 *>(out),
                       static_cast<const float2 *>(di->twiddles), log2n, (long long)batch,
                       c.problems_per_block, inverse ? -1.0f : 1.0f);
    return fail_hip(hipGetLastError(), "fft launch");
}

}  // namespace ppx
