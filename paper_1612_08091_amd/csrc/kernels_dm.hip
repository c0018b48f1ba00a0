// Density-matrix reductions: the diagonal of rho (probabilities) and the
// traces Tr(rho P) of Pauli strings.  Each touches 2^n of the 4^n entries of
// vec(rho), one strided read per entry: small next to a gate pass.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dm.hpp"

namespace qsv {
namespace dev {

template <typename R> struct VD;
template <> struct VD<double> { using T = double2; };
template <> struct VD<float> { using T = float2; };

constexpr int kDT = 256;

template <typename R>
__global__ __launch_bounds__(kDT) void k_dm_diagonal(const typename VD<R>::T *__restrict__ v,
                                                     int n, double *__restrict__ out) {
    const uint64_t dim = 1ull << n;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = (double)v[i + (i << n)].x;
}

__device__ __forceinline__ double dm_bsum(double x, double *sh) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = x;
    __syncthreads();
    x = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) x += sh[i];
    return x;
}

template <typename R>
__global__ __launch_bounds__(kDT) void k_dm_pauli(const typename VD<R>::T *__restrict__ v, int n,
                                                  const uint64_t *__restrict__ xm,
                                                  const uint64_t *__restrict__ zm,
                                                  double *__restrict__ part) {
    __shared__ double sh[8];
    const uint64_t dim = 1ull << n;
    const uint64_t x = xm[blockIdx.x], z = zm[blockIdx.x];
    double re = 0.0, im = 0.0;
    for (uint64_t r = threadIdx.x; r < dim; r += blockDim.x) {
        const auto a = v[r + ((r ^ x) << n)];
        const double sg = (__popcll(r & z) & 1) ? -1.0 : 1.0;
        re += sg * (double)a.x;
        im += sg * (double)a.y;
    }
    re = dm_bsum(re, sh);
    im = dm_bsum(im, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = re;
        part[2 * blockIdx.x + 1] = im;
    }
}

hipError_t dm_diagonal(int dtype, const void *v, int n, double *out, hipStream_t s) {
    const uint64_t dim = 1ull << n;
    const dim3 g((unsigned)std::min<uint64_t>((dim + kDT - 1) / kDT, 1u << 16));
    if (dtype == 0)
        hipLaunchKernelGGL(k_dm_diagonal<double>, g, dim3(kDT), 0, s, (const double2 *)v, n, out);
    else
        hipLaunchKernelGGL(k_dm_diagonal<float>, g, dim3(kDT), 0, s, (const float2 *)v, n, out);
    return hipGetLastError();
}

hipError_t dm_pauli_sums(int dtype, const void *v, int n, int nterms, const uint64_t *x,
                         const uint64_t *z, double *part, hipStream_t s) {
    if (nterms < 1) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL(k_dm_pauli<double>, dim3(nterms), dim3(kDT), 0, s, (const double2 *)v,
                           n, x, z, part);
    else
        hipLaunchKernelGGL(k_dm_pauli<float>, dim3(nterms), dim3(kDT), 0, s, (const float2 *)v, n,
                           x, z, part);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace qsv
