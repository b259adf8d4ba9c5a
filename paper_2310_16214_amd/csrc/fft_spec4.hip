// Instantiations of the FFT kernel specialised on log2 n for radix = P = 4
// (fft_device.h), for n = 16, 32 and 64, where the tuners pick that shape and
// the specialised kernel stages its global I/O through LDS (fft_staged_io).
// At n = 16 the specialisation alone takes about a tenth off the generic
// kernel's time at the tuned shape; at n = 64 and 256, without the staging,
// it measured 1% slower than the generic kernel, so larger sizes keep that.
#include "fft_device.h"

namespace ppx {

template <bool S>
static const void *spec4(int log2n) {
    switch (log2n) {
        case 4: return reinterpret_cast<const void *>(&k_fft_n<4, 4, S, 4>);
        case 5: return reinterpret_cast<const void *>(&k_fft_n<4, 4, S, 5>);
        case 6: return reinterpret_cast<const void *>(&k_fft_n<4, 4, S, 6>);
        default: return nullptr;
    }
}

const void *fft_spec4_kernel(int log2n, bool split) { return split ? spec4<true>(log2n) : spec4<false>(log2n); }

}  // namespace ppx
