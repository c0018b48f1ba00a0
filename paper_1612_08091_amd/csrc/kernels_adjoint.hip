// Kernels of the adjoint gradient of <H> (Jones and Gacon, 2020): the
// Pauli-sum action phi = H psi, the real inner product Re<a|b>, and a fused
// reverse step for a rotation gate exp(-i theta P / 2) that accumulates
// Im<phi|P|psi> and applies the inverse rotation to psi and phi in one pass.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"

namespace qsv {
namespace dev {

template <typename R> struct VA;
template <> struct VA<double> { using T = double2; };
template <> struct VA<float> { using T = float2; };

constexpr int kAT = 256;
constexpr int kAdjBlocks = 1024;

__device__ __forceinline__ double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double bsum(double v, double *sh) {
    v = wsum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (w == 0) {
        v = (lane < (int)(blockDim.x >> 6)) ? sh[lane] : 0.0;
        v = wsum(v);
    }
    return v;
}

// phi_j = sum_t c_t i^{ny_t} (-1)^{popcount((j ^ x_t) & z_t)} psi_{j ^ x_t}
// (P|i> = i^{ny} (-1)^{popcount(i & z)} |i ^ x>).  Terms sorted by X mask
// share their gathers.
template <typename R>
__global__ __launch_bounds__(kAT) void k_ham_apply(const typename VA<R>::T *__restrict__ psi,
                                                   typename VA<R>::T *__restrict__ phi,
                                                   uint64_t dim, int nterms,
                                                   const uint64_t *__restrict__ xm,
                                                   const uint64_t *__restrict__ zm,
                                                   const double *__restrict__ cf,
                                                   const int32_t *__restrict__ ny) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < dim;
         j += (uint64_t)gridDim.x * blockDim.x) {
        double ar = 0.0, ai = 0.0;
        // terms with equal X masks read the same amplitude: one load each run
        uint64_t lastx = ~0ull, i = 0;
        typename VA<R>::T a;
        for (int t = 0; t < nterms; ++t) {
            if (xm[t] != lastx) {
                lastx = xm[t];
                i = j ^ lastx;
                a = psi[i];
            }
            double vr = a.x, vi = a.y;
            if (__popcll(i & zm[t]) & 1) {
                vr = -vr;
                vi = -vi;
            }
            switch (ny[t] & 3) {   // multiply by i^{ny}
            case 1: { const double tmp = vr; vr = -vi; vi = tmp; } break;
            case 2: vr = -vr; vi = -vi; break;
            case 3: { const double tmp = vr; vr = vi; vi = -tmp; } break;
            default: break;
            }
            ar += cf[t] * vr;
            ai += cf[t] * vi;
        }
        typename VA<R>::T o;
        o.x = (R)ar;
        o.y = (R)ai;
        phi[j] = o;
    }
}

template <typename R>
__global__ __launch_bounds__(kAT) void k_dot_re(const typename VA<R>::T *__restrict__ a,
                                                const typename VA<R>::T *__restrict__ b,
                                                uint64_t dim, double *partial) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const auto x = a[i], y = b[i];
        acc += (double)x.x * y.x + (double)x.y * y.y;
    }
    acc = bsum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kAT) void k_sum_partials(const double *partial, int nblocks,
                                                      double *out) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += partial[b];
    acc = bsum(acc, sh);
    if (threadIdx.x == 0) *out = acc;
}

__device__ __forceinline__ uint64_t expand_ia(uint64_t g, const IndexArgs &ia) {
    for (int i = 0; i < ia.npos; ++i) {
        const uint64_t lowm = (1ull << ia.pos[i]) - 1;
        g = ((g & ~lowm) << 1) | (g & lowm);
    }
    return g | ia.ones;
}

// P applied to the pair (v0, v1) of amplitudes with target bit 0 / 1.
template <typename T>
__device__ __forceinline__ void pauli_pair(int axis, const T &v0, const T &v1, T &p0, T &p1) {
    if (axis == 1) {          // X
        p0 = v1;
        p1 = v0;
    } else if (axis == 2) {   // Y: Y|0> = i|1>, Y|1> = -i|0>
        p0.x = v1.y;
        p0.y = -v1.x;         // -i * v1
        p1.x = -v0.y;
        p1.y = v0.x;          // i * v0
    } else {                  // Z
        p0 = v0;
        p1.x = -v1.x;
        p1.y = -v1.y;
    }
}

// One reverse step of the adjoint method for U = exp(-i theta P / 2) on the
// pairs selected by ia (target bit 0, controls 1), partner offset toff:
// partial += Im sum conj(phi) P psi over the pairs, then
// psi <- U^dag psi, phi <- U^dag phi with U^dag = cos(theta/2) + i sin(theta/2) P.
template <typename R>
__global__ __launch_bounds__(kAT) void k_adj_rot(typename VA<R>::T *__restrict__ psi,
                                                 typename VA<R>::T *__restrict__ phi,
                                                 uint64_t npairs, IndexArgs ia, uint64_t toff,
                                                 int axis, double c, double s, double *partial) {
    using T = typename VA<R>::T;
    __shared__ double sh[16];
    double acc = 0.0;
    const R cr = (R)c, sr = (R)s;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < npairs;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i0 = expand_ia(g, ia), i1 = i0 + toff;
        const T a0 = psi[i0], a1 = psi[i1], f0 = phi[i0], f1 = phi[i1];
        T pa0, pa1, pf0, pf1;
        pauli_pair(axis, a0, a1, pa0, pa1);
        pauli_pair(axis, f0, f1, pf0, pf1);
        // Im(conj(f) * pa) = f.x * pa.y - f.y * pa.x
        acc += (double)f0.x * pa0.y - (double)f0.y * pa0.x + (double)f1.x * pa1.y -
               (double)f1.y * pa1.x;
        T n;
        // c v + i s (P v):  i (x + iy) = -y + ix
        n.x = cr * a0.x - sr * pa0.y;
        n.y = cr * a0.y + sr * pa0.x;
        psi[i0] = n;
        n.x = cr * a1.x - sr * pa1.y;
        n.y = cr * a1.y + sr * pa1.x;
        psi[i1] = n;
        n.x = cr * f0.x - sr * pf0.y;
        n.y = cr * f0.y + sr * pf0.x;
        phi[i0] = n;
        n.x = cr * f1.x - sr * pf1.y;
        n.y = cr * f1.y + sr * pf1.x;
        phi[i1] = n;
    }
    acc = bsum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Row sums of the partials, one workgroup per rotation, written in place to
// the row's first entry.
__global__ __launch_bounds__(kAT) void k_grad_rows(double *partial, int nb) {
    __shared__ double sh[16];
    double *row = partial + (size_t)blockIdx.x * nb;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += row[b];
    acc = bsum(acc, sh);
    if (threadIdx.x == 0) row[0] = acc;
}

// grad[param[g]] += row sum g, for the ng rotations in reverse gate order
// (one thread: a fixed summation order for parameters shared by gates).
__global__ void k_grad_finish(const double *partial, int ng, int nb, const int32_t *param,
                              double *grad, int nparams) {
    if (threadIdx.x != 0) return;
    for (int p = 0; p < nparams; ++p) grad[p] = 0.0;
    for (int g = 0; g < ng; ++g) grad[param[g]] += partial[(size_t)g * nb];
}

static unsigned adj_grid(uint64_t work) {
    uint64_t b = (work + kAT - 1) / kAT;
    if (b > kAdjBlocks) b = kAdjBlocks;
    return (unsigned)(b ? b : 1);
}

int adjoint_blocks(uint64_t npairs) { return (int)adj_grid(npairs); }

hipError_t ham_apply(int dtype, const void *psi, void *phi, uint64_t dim, int nterms,
                     const uint64_t *x, const uint64_t *z, const double *c, const int32_t *ny,
                     hipStream_t s) {
    const dim3 g((unsigned)std::min<uint64_t>((dim + kAT - 1) / kAT, 1ull << 20));
    if (dtype == 0)
        hipLaunchKernelGGL(k_ham_apply<double>, g, dim3(kAT), 0, s, (const double2 *)psi,
                           (double2 *)phi, dim, nterms, x, z, c, ny);
    else
        hipLaunchKernelGGL(k_ham_apply<float>, g, dim3(kAT), 0, s, (const float2 *)psi,
                           (float2 *)phi, dim, nterms, x, z, c, ny);
    return hipGetLastError();
}

hipError_t dot_re(int dtype, const void *a, const void *b, uint64_t dim, double *ws,
                  double *out_dev, hipStream_t s) {
    const unsigned g = adj_grid(dim);
    if (dtype == 0)
        hipLaunchKernelGGL(k_dot_re<double>, dim3(g), dim3(kAT), 0, s, (const double2 *)a,
                           (const double2 *)b, dim, ws);
    else
        hipLaunchKernelGGL(k_dot_re<float>, dim3(g), dim3(kAT), 0, s, (const float2 *)a,
                           (const float2 *)b, dim, ws);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kAT), 0, s, ws, (int)g, out_dev);
    return hipGetLastError();
}

hipError_t adjoint_rotation(int dtype, void *psi, void *phi, uint64_t npairs,
                            const IndexArgs &ia, uint64_t toff, int axis, double c, double sn,
                            double *partial, int nb, hipStream_t s) {
    // nb workgroups whatever npairs is: every entry of the row is written
    if (nb < 1) return hipErrorInvalidValue;
    const unsigned g = (unsigned)nb;
    if (dtype == 0)
        hipLaunchKernelGGL(k_adj_rot<double>, dim3(g), dim3(kAT), 0, s, (double2 *)psi,
                           (double2 *)phi, npairs, ia, toff, axis, c, sn, partial);
    else
        hipLaunchKernelGGL(k_adj_rot<float>, dim3(g), dim3(kAT), 0, s, (float2 *)psi,
                           (float2 *)phi, npairs, ia, toff, axis, c, sn, partial);
    return hipGetLastError();
}

hipError_t grad_finish(double *partial, int ng, int nb, const int32_t *param, double *grad,
                       int nparams, hipStream_t s) {
    if (ng > 0) hipLaunchKernelGGL(k_grad_rows, dim3(ng), dim3(kAT), 0, s, partial, nb);
    hipLaunchKernelGGL(k_grad_finish, dim3(1), dim3(64), 0, s, partial, ng, nb, param, grad,
                       nparams);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace qsv
