// FFT families of the mixed launch: persistent kernels whose tiles run the
// log2 n-specialised stage sequence of the job's tuned (radix = P) shape,
// with its exchange (complex values, or real and imaginary parts in turn).
// 256-thread workgroups take the shapes with at most 256 threads per problem
// (P in {4, 8, 16}); 1024-thread workgroups the larger ones (n >= 4096), one
// family for P = 8 and one for P = 16 (P = 8 needs half the LDS and fewer
// registers, so two of its workgroups fit a CU).  Each tile runs the same function as the single-call kernel
// of its shape (fft_group_ct), and the two give the same bits; the exchange
// is part of the shape because it changes how the compiler contracts the
// butterflies' products and sums into fused multiply-adds (a tile with the
// split exchange differs in the last bits from the single call with the
// complex one).
#include "fft_device.h"
#include "mixed.h"

namespace ppx {

// Whether shape (LOG2N, P, SPLIT) belongs to family FAM.
template <int FAM>
constexpr bool mix_fft_member(int log2n, int P, bool) {
    if (log2n < 4 || log2n > kFftLog2NMax || (1 << log2n) < P) return false;
    const int T = (1 << log2n) / P;
    if (FAM == kFamFft256) return T <= 256;
    return P == (FAM == kFamFft1024P8 ? 8 : 16) && T > 256 && T <= 1024;
}

template <int FAM, int ID>
__device__ __forceinline__ void mix_fft_dispatch(const MixJob &j, long long first, int count,
                                                 const float2 *__restrict__ tw, void *lds, int tx, int nt) {
    if constexpr (ID < kMixFftShapes) {
        constexpr int LOG2N = ID / 6;
        constexpr int P = 4 << ((ID / 2) % 3);
        constexpr bool SPLIT = (ID & 1) != 0;
        if constexpr (mix_fft_member<FAM>(LOG2N, P, SPLIT)) {
            static_assert(mix_fft_shape(LOG2N, P, SPLIT) == ID, "shape code");
            if (j.shape == ID) {
                fft_group_ct<P, P, SPLIT, LOG2N>(static_cast<const float2 *>(j.p[0]), static_cast<float2 *>(j.out),
                                                 tw, first, count, (j.flags & 1) ? -1.0f : 1.0f, lds, tx, nt);
                return;
            }
        }
        mix_fft_dispatch<FAM, ID + 1>(j, first, count, tw, lds, tx, nt);
    }
}

template <int FAM, bool ARGS>
__global__ __launch_bounds__(mix_block(FAM)) void k_mix_fft(MixArgs a, const float2 *tw) {
    extern __shared__ float4 lds[];
    mix_tile_loop<FAM, ARGS>(a, [&](const MixJob &j, long long first, int count, int tx, int nt) {
        mix_fft_dispatch<FAM, 0>(j, first, count, tw, lds, tx, nt);
    });
}

template <bool ARGS>
static const void *fft_kernel(int fam) {
    if (fam == kFamFft256) return reinterpret_cast<const void *>(&k_mix_fft<kFamFft256, ARGS>);
    if (fam == kFamFft1024) return reinterpret_cast<const void *>(&k_mix_fft<kFamFft1024, ARGS>);
    if (fam == kFamFft1024P8) return reinterpret_cast<const void *>(&k_mix_fft<kFamFft1024P8, ARGS>);
    return nullptr;
}

const void *mix_fft_kernel(int fam, bool args) {
    return args ? fft_kernel<true>(fam) : fft_kernel<false>(fam);
}

}  // namespace ppx
