// Tuners over the launch-parameter space (Sec. IV of arXiv:2310.16214).
#include <cstring>

#include "ppx_internal.h"

namespace ppx {

int analytical_config(int op, int dtype, int64_t n, int64_t, ppx_config &c) {
    // Provisional rule until the occupancy-model engine lands: the largest
    // radix with P = radix, and a workgroup of about 256 threads.
    std::memset(&c, 0, sizeof c);
    const int R = op == PPX_OP_FFT ? (n >= 16 ? 16 : (int)n) : 2;
    int P = op == PPX_OP_FFT ? R : 4;
    for (int L = 256; L >= 64; L /= 2) {
        for (int G = 1; G <= 16; G *= 2) {
            if (n * G != (int64_t)P * L) continue;
            c.radix = R;
            c.threads_per_block = L;
            c.problems_per_block = G;
            c.algo = 0;
            complete_config(op, dtype, n, c);
            if (validate_config(op, dtype, n, c) == PPX_OK) return PPX_OK;
            if (op == PPX_OP_FFT) {
                c.algo = PPX_FFT_LDS_SPLIT;
                c.lds_elems = 0;
                complete_config(op, dtype, n, c);
                if (validate_config(op, dtype, n, c) == PPX_OK) return PPX_OK;
            }
        }
    }
    return default_config(op, dtype, n, c);
}

}  // namespace ppx

extern "C" int tune(int, int, int64_t, int64_t, int, int, ppx_config *, double *, int *) {
    return ppx::fail(PPX_EINVAL, "tune: not available in this build");
}
