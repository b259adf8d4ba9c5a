// Tridiagonal families of the mixed launch: persistent kernels whose tiles
// run the job's tuned solver.  Systems that fit a wave (n / P <= 64) run the
// in-wave variants (the CR -> PCR hybrid, CR, PCR with shuffles or with the
// LDS exchange, Wang & Mou, Ladner-Fischer) in 256-thread workgroups, one
// kernel per dtype and per
// register tier: a kernel's VGPR count is the maximum over its shapes, and
// the P = 16 solvers (and in float32 also the PCR ones, 94-100 VGPRs against
// 56-62 for CR, WM and LF) would otherwise halve the others' occupancy.
// Larger systems run the LDS CR or PCR in 1024-thread workgroups with
// 128 KiB of LDS.
#include "mixed.h"
#include "tridiag_device.h"
#include "tridiag_wave_device.h"

namespace ppx {

template <int FAM>
using TriwType = typename std::conditional<FAM == kFamTriW32 || FAM == kFamTriW32H, float, double>::type;
// Whether the family FAM holds the in-wave shape (ALGO, P).
template <int FAM>
constexpr bool triw_member(int algo, int P) {
    return mix_triw_family(FAM == kFamTriW64 || FAM == kFamTriW64H, algo, P) == FAM;
}

template <int FAM, int ID>
__device__ __forceinline__ void mix_triw_dispatch(const MixJob &j, long long first, int count, void *smem, int tx) {
    if constexpr (ID < kMixTriwShapes) {
        using T = TriwType<FAM>;
        constexpr int ALGO = PPX_TRI_CR_PCR + ID / 4;
        constexpr int LP = ID % 4 + 1;
        constexpr int P = 1 << LP;
        if constexpr (triw_member<FAM>(ALGO, P)) {
            static_assert(mix_triw_shape(ALGO, LP) == ID, "shape code");
            if (j.shape == ID) {
                tridiag_wave_block<T, ALGO, P>(static_cast<const T *>(j.p[0]), static_cast<const T *>(j.p[1]),
                                               static_cast<const T *>(j.p[2]), static_cast<const T *>(j.p[3]),
                                               static_cast<T *>(j.out), j.log2n, first, count,
                                               static_cast<T *>(smem), tx);
                return;
            }
        }
        mix_triw_dispatch<FAM, ID + 1>(j, first, count, smem, tx);
    }
}

// float64 with 16 equations per lane: at least three waves per SIMD, as for
// the single-call kernels of those shapes (tri_wave_min_waves).
template <int FAM>
constexpr int triw_min_waves() { return FAM == kFamTriW64H ? 3 : 1; }

template <int FAM, bool ARGS>
__global__ __launch_bounds__(256, triw_min_waves<FAM>()) void k_mix_triw(MixArgs a, const float2 *) {
    extern __shared__ float4 smem[];  // PPX_TRI_PCR_REG exchange buffers, one per wave
    mix_tile_loop<FAM, ARGS>(a, [&](const MixJob &j, long long first, int count, int tx, int nt) {
        mix_triw_dispatch<FAM, 0>(j, first, count, smem, tx);
    });
}

template <bool ARGS>
__global__ __launch_bounds__(1024) void k_mix_tril(MixArgs a, const float2 *) {
    extern __shared__ float4 smem[];
    mix_tile_loop<kFamTriLds, ARGS>(a, [&](const MixJob &j, long long first, int count, int tx, int nt) {
        switch (j.shape) {
            case mix_tril_shape(false, false):
                tridiag_block<float, PPX_TRI_CR>(static_cast<const float *>(j.p[0]), static_cast<const float *>(j.p[1]),
                                                 static_cast<const float *>(j.p[2]), static_cast<const float *>(j.p[3]),
                                                 static_cast<float *>(j.out), j.log2n, first, count,
                                                 reinterpret_cast<float *>(smem));
                break;
            case mix_tril_shape(false, true):
                tridiag_block<float, PPX_TRI_PCR>(static_cast<const float *>(j.p[0]), static_cast<const float *>(j.p[1]),
                                                  static_cast<const float *>(j.p[2]), static_cast<const float *>(j.p[3]),
                                                  static_cast<float *>(j.out), j.log2n, first, count,
                                                  reinterpret_cast<float *>(smem));
                break;
            case mix_tril_shape(true, false):
                tridiag_block<double, PPX_TRI_CR>(static_cast<const double *>(j.p[0]), static_cast<const double *>(j.p[1]),
                                                  static_cast<const double *>(j.p[2]), static_cast<const double *>(j.p[3]),
                                                  static_cast<double *>(j.out), j.log2n, first, count,
                                                  reinterpret_cast<double *>(smem));
                break;
            default:
                tridiag_block<double, PPX_TRI_PCR>(static_cast<const double *>(j.p[0]), static_cast<const double *>(j.p[1]),
                                                   static_cast<const double *>(j.p[2]), static_cast<const double *>(j.p[3]),
                                                   static_cast<double *>(j.out), j.log2n, first, count,
                                                   reinterpret_cast<double *>(smem));
                break;
        }
    });
}

// The hybrid across waves: a tile is nt / (n / P) systems (nt the workgroup
// size), the lanes exchanging through LDS slots (two sets of a, c, d per
// thread).
template <int FAM, int LP>
__device__ __forceinline__ void mix_trib_dispatch(const MixJob &j, long long first, int count, void *smem, int tx,
                                                  int nt) {
    if constexpr (LP <= 4) {
        using T = typename std::conditional<FAM == kFamTriBlk32 || FAM == kFamTriBlk32H, float, double>::type;
        constexpr int P = 1 << LP;
        if constexpr ((FAM == kFamTriBlk32H || FAM == kFamTriBlk64H) == (P == 16)) {
            if (j.shape == LP - 1) {
                tridiag_blk_block<T, P>(static_cast<const T *>(j.p[0]), static_cast<const T *>(j.p[1]),
                                        static_cast<const T *>(j.p[2]), static_cast<const T *>(j.p[3]),
                                        static_cast<T *>(j.out), j.log2n, first, count, static_cast<T *>(smem), tx,
                                        nt);
                return;
            }
        }
        mix_trib_dispatch<FAM, LP + 1>(j, first, count, smem, tx, nt);
    }
}

template <int FAM, bool ARGS>
__global__ __launch_bounds__(mix_block(FAM)) void k_mix_trib(MixArgs a, const float2 *) {
    extern __shared__ float4 smem[];
    mix_tile_loop<FAM, ARGS>(a, [&](const MixJob &j, long long first, int count, int tx, int nt) {
        mix_trib_dispatch<FAM, 1>(j, first, count, smem, tx, nt);
    });
}

template <bool ARGS>
static const void *tri_kernel(int fam) {
    switch (fam) {
        case kFamTriW32: return reinterpret_cast<const void *>(&k_mix_triw<kFamTriW32, ARGS>);
        case kFamTriW32H: return reinterpret_cast<const void *>(&k_mix_triw<kFamTriW32H, ARGS>);
        case kFamTriW64: return reinterpret_cast<const void *>(&k_mix_triw<kFamTriW64, ARGS>);
        case kFamTriW64H: return reinterpret_cast<const void *>(&k_mix_triw<kFamTriW64H, ARGS>);
        case kFamTriLds: return reinterpret_cast<const void *>(&k_mix_tril<ARGS>);
        case kFamTriBlk32: return reinterpret_cast<const void *>(&k_mix_trib<kFamTriBlk32, ARGS>);
        case kFamTriBlk32H: return reinterpret_cast<const void *>(&k_mix_trib<kFamTriBlk32H, ARGS>);
        case kFamTriBlk64: return reinterpret_cast<const void *>(&k_mix_trib<kFamTriBlk64, ARGS>);
        case kFamTriBlk64H: return reinterpret_cast<const void *>(&k_mix_trib<kFamTriBlk64H, ARGS>);
        default: return nullptr;
    }
}

const void *mix_tri_kernel(int fam, bool args) { return args ? tri_kernel<true>(fam) : tri_kernel<false>(fam); }

}  // namespace ppx
