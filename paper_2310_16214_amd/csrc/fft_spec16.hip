// Instantiations of the FFT kernels specialised on log2 n for radix = P = 16
// (fft_device.h), in their own translation unit so they compile in parallel.
#include "fft_device.h"

namespace ppx {

using FftKernel = void (*)(const float2 *, float2 *, const float2 *, int, long long, int, float);

template <bool S, bool PIPE, int L2N>
static FftKernel spec_entry() {
    constexpr int lT = L2N - clog2(16);
    if constexpr (lT >= 0 && (1 << lT) <= fft_max_threads(16))
        return PIPE ? &k_fft_np<16, 16, S, L2N> : &k_fft_n<16, 16, S, L2N>;
    else
        return nullptr;
}

template <bool S, bool PIPE>
static FftKernel spec_sizes(int log2n) {
    switch (log2n) {
        case 4: return spec_entry<S, PIPE, 4>();
        case 5: return spec_entry<S, PIPE, 5>();
        case 6: return spec_entry<S, PIPE, 6>();
        case 7: return spec_entry<S, PIPE, 7>();
        case 8: return spec_entry<S, PIPE, 8>();
        case 9: return spec_entry<S, PIPE, 9>();
        case 10: return spec_entry<S, PIPE, 10>();
        case 11: return spec_entry<S, PIPE, 11>();
        case 12: return spec_entry<S, PIPE, 12>();
        case 13: return spec_entry<S, PIPE, 13>();
        case 14: return spec_entry<S, PIPE, 14>();
        default: return nullptr;
    }
}

const void *fft_spec16_kernel(int log2n, bool split, bool pipe) {
    FftKernel k = split ? (pipe ? spec_sizes<true, true>(log2n) : spec_sizes<true, false>(log2n))
                        : (pipe ? spec_sizes<false, true>(log2n) : spec_sizes<false, false>(log2n));
    return reinterpret_cast<const void *>(k);
}

}  // namespace ppx
