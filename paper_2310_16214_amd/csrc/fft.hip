// Host launcher of the kernels in fft_device.h.
#include "fft_device.h"

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

int64_t fft_lds_bytes(int n, int gb, int algo) {
    return (int64_t)gb * n * (algo == PPX_FFT_LDS_SPLIT ? 4 : 8);
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

static FftKernel fft_lookup(int radix, int P, int algo) {
    return algo == PPX_FFT_LDS_SPLIT ? fft_lookup_s<true>(radix, P) : fft_lookup_s<false>(radix, P);
}

const void *fft_kernel(int radix, int P, int algo) {
    return reinterpret_cast<const void *>(fft_lookup(radix, P, algo));
}

int launch_fft(const void *in, void *out, int log2n, int64_t batch, const ppx_config &c,
               bool inverse, hipStream_t s) {
    const DeviceInfo *di = device_info();
    if (!di) return PPX_EDEVICE;
    FftKernel k = fft_lookup(c.radix, c.elems_per_thread, c.algo);
    if (!k) return fail(PPX_ECONFIG, "no FFT kernel for this radix / elements-per-thread");
    const int n = 1 << log2n;
    const int64_t lds = fft_lds_bytes(n, c.problems_per_block, c.algo);
    if (lds > di->lds_per_block) return fail(PPX_ECONFIG, "FFT configuration exceeds the LDS per workgroup");
    const int64_t grid = (batch + c.problems_per_block - 1) / c.problems_per_block;
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(c.threads_per_block), (size_t)lds, s,
                       static_cast<const float2 *>(in), static_cast<float2 *>(out),
                       static_cast<const float2 *>(di->twiddles), log2n, (long long)batch,
                       c.problems_per_block, inverse ? -1.0f : 1.0f);
    return fail_hip(hipGetLastError(), "fft launch");
}

}  // namespace ppx
