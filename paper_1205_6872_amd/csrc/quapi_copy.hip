// Device copy used to measure the attainable HBM read+write rate of the GPU
// (the ceiling that the step kernels are compared with).  Each block copies
// one contiguous chunk with 16-byte accesses, a few loads in flight per
// thread before their stores.  Not part of the propagation path.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "quapi.h"

namespace {

constexpr int kCopyBlock = 512;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;

template <bool NT>
__global__ __launch_bounds__(kCopyBlock) void copy_chunks_kernel(const u32x4 *__restrict__ src,
                                                                 u32x4 *__restrict__ dst, size_t n16,
                                                                 size_t chunk16) {
    const size_t base = (size_t)blockIdx.x * chunk16;
    const size_t end = base + chunk16 < n16 ? base + chunk16 : n16;
    for (size_t i = base + threadIdx.x; i < end; i += (size_t)kCopyBlock * kCopyUnroll) {
        u32x4 v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const size_t k = i + (size_t)u * kCopyBlock;
            if (k < end) v[u] = NT ? __builtin_nontemporal_load(src + k) : src[k];
        }
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const size_t k = i + (size_t)u * kCopyBlock;
            if (k < end) dst[k] = v[u];
        }
    }
}

}  // namespace

extern "C" quapi_status quapi_copy_bandwidth(const void *src, void *dst, size_t bytes, size_t chunk_bytes,
                                             int nontemporal, void *hip_stream) {
    if (!src || !dst || bytes == 0 || bytes % 16 != 0 || chunk_bytes < 16 * kCopyBlock ||
        chunk_bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(dst) % 16 != 0)
        return QUAPI_ERR_INVALID;
    const size_t n16 = bytes / 16, chunk16 = chunk_bytes / 16;
    const size_t blocks = (n16 + chunk16 - 1) / chunk16;
    if (blocks > 0x7fffffffu) return QUAPI_ERR_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    if (nontemporal)
        hipLaunchKernelGGL(copy_chunks_kernel<true>, dim3((unsigned)blocks), dim3(kCopyBlock), 0, st,
                           (const u32x4 *)src, (u32x4 *)dst, n16, chunk16);
    else
        hipLaunchKernelGGL(copy_chunks_kernel<false>, dim3((unsigned)blocks), dim3(kCopyBlock), 0, st,
                           (const u32x4 *)src, (u32x4 *)dst, n16, chunk16);
    return hipGetLastError() == hipSuccess ? QUAPI_OK : QUAPI_ERR_DEVICE;
}
