// Copy-bandwidth probe: a streaming device-to-device copy, the practical
// ceiling of a pass that reads and writes every byte once (the roofline of
// the state-vector passes is HBM bandwidth).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"

namespace qsv {
namespace dev {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Each workgroup moves contiguous blocks of 256 x 8 sixteen-byte elements,
// the eight loads of a thread in flight together, with nontemporal loads and
// stores (the data is not reused).  Of the shapes measured (grid-strided or
// blocked, 4-16 elements per thread, 4-64 workgroups per compute unit) this
// one is the fastest over 16 GiB.
__global__ __launch_bounds__(256) void k_copy16(const u32x4 *__restrict__ src,
                                               u32x4 *__restrict__ dst, uint64_t n16) {
    constexpr uint64_t kBlock = 256ull * 8;
    for (uint64_t b0 = (uint64_t)blockIdx.x * kBlock; b0 < n16; b0 += (uint64_t)gridDim.x * kBlock) {
        u32x4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint64_t i = b0 + (uint64_t)u * 256 + threadIdx.x;
            if (i < n16) v[u] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint64_t i = b0 + (uint64_t)u * 256 + threadIdx.x;
            if (i < n16) __builtin_nontemporal_store(v[u], dst + i);
        }
    }
}

hipError_t copy_probe(const void *src, void *dst, uint64_t bytes, hipStream_t s) {
    if (bytes % 16) return hipErrorInvalidValue;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const uint64_t n16 = bytes / 16;
    const uint64_t want = (n16 + 2047) / 2048;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)cus * 64));
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, s, (const u32x4 *)src, (u32x4 *)dst, n16);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace qsv
