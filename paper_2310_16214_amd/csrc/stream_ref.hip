// Streaming reference kernel (ppx_stream_reference in ppx_tune.h): k input
// arrays summed into one output with 16-byte accesses, one per thread, the
// output stored non-temporally like the library's results.  It moves the
// same HBM bytes as a batched call with k input streams, so its rate is the
// practical ceiling for that call size and pattern.
#include <hip/hip_runtime.h>

#include "device.h"

#include "ppx_internal.h"
#include "ppx_tune.h"

namespace ppx {

template <int K>
__global__ __launch_bounds__(256) void k_stream(const float4 *__restrict__ a, const float4 *__restrict__ b,
                                                const float4 *__restrict__ c, const float4 *__restrict__ d,
                                                float4 *__restrict__ x, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 v = a[i];
    if constexpr (K >= 2) {
        const float4 w = b[i];
        v = make_float4(v.x + w.x, v.y + w.y, v.z + w.z, v.w + w.w);
    }
    if constexpr (K >= 3) {
        const float4 w = c[i];
        v = make_float4(v.x + w.x, v.y + w.y, v.z + w.z, v.w + w.w);
    }
    if constexpr (K >= 4) {
        const float4 w = d[i];
        v = make_float4(v.x + w.x, v.y + w.y, v.z + w.z, v.w + w.w);
    }
    __builtin_nontemporal_store(__builtin_bit_cast(u32x4, v), reinterpret_cast<u32x4 *>(x + i));
}

}  // namespace ppx

using namespace ppx;

extern "C" int ppx_stream_reference(const void *const *in, int k, void *out, int64_t bytes, void *stream) {
    if (!in || !out || k < 1 || k > 4) return fail(PPX_EINVAL, "stream reference: 1..4 inputs and an output");
    if (bytes <= 0 || bytes % 16 != 0 || bytes > (int64_t(1) << 36))
        return fail(PPX_EINVAL, "stream reference: bytes must be a positive multiple of 16, at most 2^36");
    for (int i = 0; i < k; ++i)
        if (!in[i] || reinterpret_cast<uintptr_t>(in[i]) % 16 != 0)
            return fail(PPX_EINVAL, "stream reference: inputs must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(out) % 16 != 0) return fail(PPX_EINVAL, "stream reference: output alignment");
    if (!device_info()) return PPX_EDEVICE;
    const long long n4 = bytes / 16;
    const dim3 grid((unsigned)((n4 + 255) / 256)), block(256);
    const float4 *p[4];
    for (int i = 0; i < 4; ++i) p[i] = static_cast<const float4 *>(in[i < k ? i : 0]);
    hipStream_t s = static_cast<hipStream_t>(stream);
    float4 *x = static_cast<float4 *>(out);
    switch (k) {
        case 1: hipLaunchKernelGGL(k_stream<1>, grid, block, 0, s, p[0], p[1], p[2], p[3], x, n4); break;
        case 2: hipLaunchKernelGGL(k_stream<2>, grid, block, 0, s, p[0], p[1], p[2], p[3], x, n4); break;
        case 3: hipLaunchKernelGGL(k_stream<3>, grid, block, 0, s, p[0], p[1], p[2], p[3], x, n4); break;
        default: hipLaunchKernelGGL(k_stream<4>, grid, block, 0, s, p[0], p[1], p[2], p[3], x, n4); break;
    }
    const int rc = fail_hip(hipGetLastError(), "stream reference launch");
    if (rc == PPX_OK) fail(PPX_OK, "");
    return rc;
}
