// Device-side building blocks for the gfx950 kernels: complex arithmetic,
// radix-R DFTs held in registers, and wave64 lane networks for scans.
#pragma once

#include <hip/hip_runtime.h>

namespace ppx {

// ------------------------------------------------------------------ complex
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// cos and sin of 2*pi*e/16 for the odd sixteenths (the even ones are handled
// by exact special cases below).
__host__ __device__ constexpr float cos16(int e) {
    return e == 1 ? 0.92387953251128674f : e == 3 ? 0.38268343236508978f
         : e == 5 ? -0.38268343236508978f : e == 7 ? -0.92387953251128674f : 0.0f;
}
__host__ __device__ constexpr float sin16(int e) {
    return (e == 1 || e == 7) ? 0.38268343236508978f
         : (e == 3 || e == 5) ? 0.92387953251128674f : 0.0f;
}
constexpr float kHalfSqrt2 = 0.70710678118654752f;

// x * exp(-2*pi*i*m/M) for M a power of two <= 16 and m < M/2, with the
// multiplications by 1, -i and (+-1 - i)/sqrt(2) done exactly as adds/swaps.
template <int M, int m>
__host__ __device__ __forceinline__ float2 twiddle_const(float2 x) {
    constexpr int e = m * (16 / M);  // angle in sixteenths of a turn, 0..7
    if constexpr (e == 0) {
        return x;
    } else if constexpr (e == 4) {
        return make_float2(x.y, -x.x);
    } else if constexpr (e == 2) {
        return make_float2(kHalfSqrt2 * (x.x + x.y), kHalfSqrt2 * (x.y - x.x));
    } else if constexpr (e == 6) {
        return make_float2(kHalfSqrt2 * (x.y - x.x), -kHalfSqrt2 * (x.x + x.y));
    } else {
        constexpr float c = cos16(e), s = sin16(e);
        return make_float2(x.x * c + x.y * s, x.y * c - x.x * s);
    }
}

// In-register forward DFT of length M (power of two <= 16), natural order in
// and out: u[k] <- sum_j u[j] exp(-2 pi i j k / M).  Radix-2 decimation in
// time, fully unrolled; the even/odd split is pure register renaming.
template <int M, int k>
__host__ __device__ __forceinline__ void dft_combine(float2 (&u)[M], const float2 (&e)[M / 2],
                                            const float2 (&o)[M / 2]) {
    if constexpr (k < M / 2) {
        const float2 t = twiddle_const<M, k>(o[k]);
        u[k] = cadd(e[k], t);
        u[k + M / 2] = csub(e[k], t);
        dft_combine<M, k + 1>(u, e, o);
    }
}

template <int M>
struct RegDFT {
    __host__ __device__ __forceinline__ static void run(float2 (&u)[M]) {
        float2 e[M / 2], o[M / 2];
#pragma unroll
        for (int j = 0; j < M / 2; ++j) {
            e[j] = u[2 * j];
            o[j] = u[2 * j + 1];
        }
        RegDFT<M / 2>::run(e);
        RegDFT<M / 2>::run(o);
        dft_combine<M, 0>(u, e, o);
    }
};
template <>
struct RegDFT<1> {
    __host__ __device__ __forceinline__ static void run(float2 (&)[1]) {}
};

// ------------------------------------------------------- buffer accesses
// Raw buffer loads and stores through a descriptor: a lane whose byte offset
// falls outside the descriptor's range reads zeros and writes nothing, with
// no branch.  Used by the persistent kernels, whose per-group descriptors
// cover exactly the group's problems inside the batch.
constexpr int kBufferFlags = 0x00020000;  // word 3 of a raw buffer descriptor (32-bit data format)
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The descriptor of group `group` (gb problems of `elems` elements of `es`
// bytes each) of an array of `batch` problems.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t group_rsrc(const void *base, long long group, int gb,
                                                            long long elems, int es, long long batch) {
    const long long left = batch - group * gb;  // problems of the batch from this group on
    const int bytes = left <= 0 ? 0 : (int)((left >= gb ? gb : left) * elems * es);
    const char *p = static_cast<const char *>(base) + (left > 0 ? group * gb * elems * es : 0);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, bytes, kBufferFlags);
}

// Non-temporal stores (the nt bit of gfx950's cache-policy operand), used for
// the FFT kernels' results.  Timed inside whole benchmark steps against the
// default policy (builds alternating step by step), they take 2-6% off the
// FFT calls from n = 32 on and up to 18% off the scans that follow them (less
// dirty data left in the caches to drain), and 1.5% off the step; the first
// call of the step (n = 16) is 12% slower with them.  Repeated calls of one
// kernel on the same buffers show larger gains (n = 16384: 112 -> 95 us), part
// of which is the input staying cached between the calls.  The scan and
// tridiagonal kernels keep the default policy: with the hint they measured
// neutral to 33% slower per call (worst where each lane stores a contiguous
// chunk, so that one store instruction covers only part of each line) and the
// step no faster.  Loads keep the default policy: on a plain copy, hinting
// both directions was slower than hinting the stores alone.
constexpr int kStoreNT = 2;

__device__ __forceinline__ void store_nt(unsigned *p, unsigned v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_nt(u32x2 *p, u32x2 v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_nt(u32x4 *p, u32x4 v) { __builtin_nontemporal_store(v, p); }
// Any 4-, 8- or 16-byte value.
template <typename V>
__device__ __forceinline__ void store_nt_any(V *p, const V &v) {
    if constexpr (sizeof(V) == 16) store_nt(reinterpret_cast<u32x4 *>(p), __builtin_bit_cast(u32x4, v));
    else if constexpr (sizeof(V) == 8) store_nt(reinterpret_cast<u32x2 *>(p), __builtin_bit_cast(u32x2, v));
    else {
        static_assert(sizeof(V) == 4, "4, 8 or 16 bytes");
        store_nt(reinterpret_cast<unsigned *>(p), __builtin_bit_cast(unsigned, v));
    }
}

// K contiguous 4- or 8-byte values at byte offset voff (16-byte words where
// the size allows; the constant part of each offset in the scalar operand).
template <typename T, int K>
__device__ __forceinline__ void buf_load(T (&v)[K], __amdgpu_buffer_rsrc_t r, int voff) {
    constexpr int B = K * (int)sizeof(T);
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int w = 0; w < B / 16; ++w) {
            const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 16 * w, 0);
            __builtin_memcpy(&v[w * 16 / (int)sizeof(T)], &x, 16);
        }
    } else if constexpr (B == 8) {
        const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0);
        __builtin_memcpy(&v[0], &x, 8);
    } else {
        static_assert(B == 4, "4, 8 or a multiple of 16 bytes");
        const unsigned x = __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0);
        __builtin_memcpy(&v[0], &x, 4);
    }
}

template <typename T, int K, int POLICY = 0>
__device__ __forceinline__ void buf_store(const T (&v)[K], __amdgpu_buffer_rsrc_t r, int voff) {
    constexpr int B = K * (int)sizeof(T);
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int w = 0; w < B / 16; ++w) {
            u32x4 x;
            __builtin_memcpy(&x, &v[w * 16 / (int)sizeof(T)], 16);
            __builtin_amdgcn_raw_buffer_store_b128(x, r, voff, 16 * w, POLICY);
        }
    } else if constexpr (B == 8) {
        u32x2 x;
        __builtin_memcpy(&x, &v[0], 8);
        __builtin_amdgcn_raw_buffer_store_b64(x, r, voff, 0, POLICY);
    } else {
        static_assert(B == 4, "4, 8 or a multiple of 16 bytes");
        unsigned x;
        __builtin_memcpy(&x, &v[0], 4);
        __builtin_amdgcn_raw_buffer_store_b32(x, r, voff, 0, POLICY);
    }
}

// ------------------------------------------------------------ lane networks
// DPP controls (GFX9 encoding).
constexpr int kDppRowShr = 0x110;     // + shift (1..15), within 16-lane rows
constexpr int kDppRowBcast15 = 0x142; // lane 15 of each row -> next row
constexpr int kDppRowBcast31 = 0x143; // lane 31 -> rows 2 and 3

// A 32-bit lane operation applied to each 32-bit word of a 4- or 8-byte
// value (the cross-lane instructions move 32 bits per lane).
struct Words2 {
    int lo, hi;
};
template <typename T, typename F>
__device__ __forceinline__ T per_word(T v, F f) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, f(__builtin_bit_cast(int, v)));
    } else {
        static_assert(sizeof(T) == 8, "4- or 8-byte values");
        Words2 w = __builtin_bit_cast(Words2, v);
        w.lo = f(w.lo);
        w.hi = f(w.hi);
        return __builtin_bit_cast(T, w);
    }
}

// Value of lane (lane - 1) across the whole wave (DPP wave_shr:1); lane 0
// receives 0.  Must be called with all 64 lanes active.
constexpr int kDppWaveShr1 = 0x138;
template <typename T>
__device__ __forceinline__ T dpp_wave_shr1(T v) {
    return per_word(v, [](int x) { return __builtin_amdgcn_update_dpp(0, x, kDppWaveShr1, 0xf, 0xf, false); });
}

// Value of lane (lane - D) within the same 16-lane row, 0 where that lane is
// outside the row.
template <int D, typename T>
__device__ __forceinline__ T dpp_row_shr(T v) {
    return per_word(v, [](int x) { return __builtin_amdgcn_update_dpp(0, x, kDppRowShr + D, 0xf, 0xf, false); });
}

// Inclusive scan over aligned segments of SEG lanes (SEG power of two <= 64),
// Kogge-Stone shape: shifts 1, 2, 4, 8 inside rows, then the row broadcasts.
// Must be called with all 64 lanes active.
template <typename T>
__device__ __forceinline__ T lanes_scan_ks(T x, int seg, int lane) {
    const int ls = lane & (seg - 1);
    if (seg > 1) { T y = dpp_row_shr<1>(x); if (ls >= 1) x += y; }
    if (seg > 2) { T y = dpp_row_shr<2>(x); if (ls >= 2) x += y; }
    if (seg > 4) { T y = dpp_row_shr<4>(x); if (ls >= 4) x += y; }
    if (seg > 8) { T y = dpp_row_shr<8>(x); if (ls >= 8) x += y; }
    if (seg > 16) {
        // rows 1 and 3 receive the last lane of rows 0 and 2
        x += per_word(x, [](int w) { return __builtin_amdgcn_update_dpp(0, w, kDppRowBcast15, 0xa, 0xf, false); });
    }
    if (seg > 32) {
        // rows 2 and 3 receive lane 31
        x += per_word(x, [](int w) { return __builtin_amdgcn_update_dpp(0, w, kDppRowBcast31, 0xc, 0xf, false); });
    }
    return x;
}

// ds_swizzle in bit-mask mode within 32-lane halves: source lane =
// (lane & AND) | OR.
template <int AND, int OR, typename T>
__device__ __forceinline__ T swz(T v) {
    return per_word(v, [](int w) { return __builtin_amdgcn_ds_swizzle(w, (AND & 31) | ((OR & 31) << 5)); });
}

// Inclusive scan over aligned segments of SEG lanes, Ladner-Fischer shape
// (minimum depth: at step d every lane of the upper half of each 2d-block
// adds the last value of the lower half, fetched by a swizzle broadcast).
template <typename T>
__device__ __forceinline__ T lanes_scan_lf(T x, int seg, int lane) {
    if (seg > 1) { T y = swz<0x1e, 0x00>(x); if (lane & 1) x += y; }
    if (seg > 2) { T y = swz<0x1c, 0x01>(x); if (lane & 2) x += y; }
    if (seg > 4) { T y = swz<0x18, 0x03>(x); if (lane & 4) x += y; }
    if (seg > 8) { T y = swz<0x10, 0x07>(x); if (lane & 8) x += y; }
    if (seg > 16) { T y = swz<0x00, 0x0f>(x); if (lane & 16) x += y; }
    if (seg > 32) {
        T y = per_word(x, [](int w) { return __builtin_amdgcn_readlane(w, 31); });
        if (lane & 32) x += y;
    }
    return x;
}

}  // namespace ppx
