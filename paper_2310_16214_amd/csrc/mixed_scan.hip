// Scan families of the mixed launch: persistent kernels whose tiles run the
// job's tuned scan shape (values per thread, lane network, inclusive or
// exclusive) on whole problems of T = n/P threads: 256-thread workgroups for
// T <= 256, 1024-thread ones above.
#include "mixed.h"
#include "scan_device.h"

namespace ppx {

template <int ID, typename Wt>
__device__ __forceinline__ void mix_scan_dispatch(const MixJob &j, long long first, int count, Wt *wave_tot, int tx) {
    if constexpr (ID < kMixScanShapes) {
        constexpr int DT = ID / 10;
        constexpr int LP = (ID / 2) % 5 + 1;
        constexpr int P = 1 << LP;
        constexpr int ALGO = (ID & 1) ? PPX_SCAN_LF : PPX_SCAN_KS;
        using T = typename std::conditional<DT == PPX_I32, int, typename std::conditional<DT == PPX_F32, float, double>::type>::type;
        if constexpr (DT != PPX_F64 || P <= kScanF64MaxElems) {
            static_assert(mix_scan_shape(DT, LP, ALGO == PPX_SCAN_LF) == ID, "shape code");
            if (j.shape == ID) {
                const T *in = static_cast<const T *>(j.p[0]);
                T *out = static_cast<T *>(j.out);
                T *wt = reinterpret_cast<T *>(wave_tot);
                if (j.flags & 1) scan_block<T, P, ALGO, true>(in, out, j.log2n, first, count, wt, tx);
                else scan_block<T, P, ALGO, false>(in, out, j.log2n, first, count, wt, tx);
                return;
            }
        }
        mix_scan_dispatch<ID + 1>(j, first, count, wave_tot, tx);
    }
}

template <int FAM, bool ARGS>
__global__ __launch_bounds__(mix_block(FAM)) void k_mix_scan(MixArgs a, const float2 *) {
    __shared__ double wave_tot[mix_block(FAM) / kWave];  // int and float totals use its start
    mix_tile_loop<FAM, ARGS>(a, [&](const MixJob &j, long long first, int count, int tx, int nt) {
        mix_scan_dispatch<0>(j, first, count, wave_tot, tx);
    });
}

template <bool ARGS>
static const void *scan_kernel(int fam) {
    if (fam == kFamScan256) return reinterpret_cast<const void *>(&k_mix_scan<kFamScan256, ARGS>);
    if (fam == kFamScan1024) return reinterpret_cast<const void *>(&k_mix_scan<kFamScan1024, ARGS>);
    return nullptr;
}

const void *mix_scan_kernel(int fam, bool args) {
    return args ? scan_kernel<true>(fam) : scan_kernel<false>(fam);
}

}  // namespace ppx
