// Instantiations of the FFT kernel specialised on log2 n for radix = P = 4
// (fft_device.h), for n = 16, the smallest size the library takes.  There it
// takes about a tenth off the generic kernel's time at the tuned shape (4
// threads per problem, 64 problems per workgroup); at n = 64 and 256 it
// measured 1% slower than the generic kernel, so larger sizes keep that one.
#include "fft_device.h"

namespace ppx {

const void *fft_spec4_kernel(int log2n, bool split) {
    if (log2n != 4) return nullptr;
    return split ? reinterpret_cast<const void *>(&k_fft_n<4, 4, true, 4>)
                 : reinterpret_cast<const void *>(&k_fft_n<4, 4, false, 4>);
}

}  // namespace ppx
