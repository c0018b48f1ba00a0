// Copy-bandwidth probe: a streaming device-to-device copy, the practical
// ceiling of a pass that reads and writes every byte once (the roofline of
// the state-vector passes is HBM bandwidth).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"

namespace qsv {
namespace dev {

// Each thread moves 4 x 16 bytes per step, grid-strided; the four loads are
// in flight together.
__global__ __launch_bounds__(256) void k_copy16(const uint4 *__restrict__ src,
                                               uint4 *__restrict__ dst, uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride],
                    d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

hipError_t copy_probe(const void *src, void *dst, uint64_t bytes, hipStream_t s) {
    if (bytes % 16) return hipErrorInvalidValue;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const uint64_t n16 = bytes / 16;
    const uint64_t want = (n16 + 255) / 256;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)cus * 16));
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, s, (const uint4 *)src, (uint4 *)dst, n16);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace qsv
