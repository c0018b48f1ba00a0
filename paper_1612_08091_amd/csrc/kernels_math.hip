// Emulated math gate as one gather pass: every output amplitude reads the
// amplitude whose register value the table maps onto its own.  Writes are
// contiguous; reads follow the permutation (contiguous runs when the table
// shifts values, as AddConstant does).  One read and one write of the state
// plus 4 bytes of inverse table per amplitude, which stay in cache for small
// registers: an HBM-bound pass.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "math_gate.hpp"

namespace qsv {
namespace dev {

template <typename R> struct VM;
template <> struct VM<double> { using T = double2; };
template <> struct VM<float> { using T = float2; };

constexpr int kMT = 256;

template <typename R>
__global__ __launch_bounds__(kMT) void k_math_gather(const typename VM<R>::T *__restrict__ in,
                                                     typename VM<R>::T *__restrict__ out,
                                                     uint64_t dim, MathArgs a,
                                                     const uint32_t *__restrict__ inv) {
    const uint32_t vmask = (a.w >= 32) ? ~0u : ((1u << a.w) - 1u);
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < dim;
         j += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t src = j;
        if ((j & a.ctrl) == a.ctrl) {
            uint32_t y, x;
            uint64_t d = 0;
            if (a.shift >= 0) {
                y = (uint32_t)(j >> a.shift) & vmask;
                x = inv[y];
                d = (uint64_t)x << a.shift;
            } else {
                y = 0;
                for (int b = 0; b < a.w; ++b) y |= (uint32_t)((j >> a.pos[b]) & 1u) << b;
                x = inv[y];
                for (int b = 0; b < a.w; ++b) d |= (uint64_t)((x >> b) & 1u) << a.pos[b];
            }
            src = (j & ~a.regmask) | d;
        }
        out[j] = in[src];
    }
}

hipError_t math_gather(int dtype, const void *in, void *out, uint64_t dim, const MathArgs &a,
                       const uint32_t *inv, hipStream_t s) {
    if (a.w < 1 || a.w > kMaxMathBits || !in || !out || !inv) return hipErrorInvalidValue;
    const dim3 g((unsigned)std::min<uint64_t>((dim + kMT - 1) / kMT, 1ull << 20));
    if (dtype == 0)
        hipLaunchKernelGGL(k_math_gather<double>, g, dim3(kMT), 0, s, (const double2 *)in,
                           (double2 *)out, dim, a, inv);
    else
        hipLaunchKernelGGL(k_math_gather<float>, g, dim3(kMT), 0, s, (const float2 *)in,
                           (float2 *)out, dim, a, inv);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace qsv
