// Per-gate kernels for gfx950: one dense or monomial (permutation/diagonal)
// update streamed through HBM, one thread per group of 2^k amplitudes.
//
// Update rule (gate-level simulation, ProjectQ Sec. 4.3.2; controls on |1>,
// Sec. 4.1.3): for every index i whose target bits are 0 and whose control
// bits are 1, out[i + off(r)] = sum_c U[r][c] psi[i + off(c)].
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace qsv {
namespace dev {

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

__device__ __forceinline__ uint64_t expand_index(uint64_t g, const IndexArgs &ia) {
    for (int i = 0; i < ia.npos; ++i) {
        const int p = ia.pos[i];
        const uint64_t lowm = (1ull << p) - 1;
        g = ((g & ~lowm) << 1) | (g & lowm);
    }
    return g | ia.ones;
}

template <typename R, int D>
struct DenseArgsT {
    R mr[D * D];
    R mi[D * D];
    uint64_t off[D];
};

template <typename R>
struct MonoArgsT {
    R vr[32], vi[32];
    uint64_t off[32];
    uint64_t srcoff[32];
    uint32_t touch;
};

// ------------------------------------------------------------- per gate
template <typename R, int K>
__global__ __launch_bounds__(256) void k_dense(typename V2<R>::T *__restrict__ psi,
                                               uint64_t ngroups, IndexArgs ia,
                                               DenseArgsT<R, (1 << K)> a) {
    using T = typename V2<R>::T;
    constexpr int D = 1 << K;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t base = expand_index(g, ia);
        T x[D];
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = psi[base + a.off[c]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            R yr = 0, yi = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const R mr = a.mr[r * D + c], mi = a.mi[r * D + c];
                yr += mr * x[c].x - mi * x[c].y;
                yi += mr * x[c].y + mi * x[c].x;
            }
            T y;
            y.x = yr;
            y.y = yi;
            psi[base + a.off[r]] = y;
        }
    }
}

template <typename R, int K>
__global__ __launch_bounds__(256) void k_mono(typename V2<R>::T *__restrict__ psi,
                                              uint64_t ngroups, IndexArgs ia, MonoArgsT<R> a) {
    using T = typename V2<R>::T;
    constexpr int D = 1 << K;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t base = expand_index(g, ia);
        T y[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            if ((a.touch >> r) & 1) {
                const T s = psi[base + a.srcoff[r]];
                y[r].x = a.vr[r] * s.x - a.vi[r] * s.y;
                y[r].y = a.vr[r] * s.y + a.vi[r] * s.x;
            }
        }
#pragma unroll
        for (int r = 0; r < D; ++r)
            if ((a.touch >> r) & 1) psi[base + a.off[r]] = y[r];
    }
}

// The per-gate kernels stride over their groups; 2^20 blocks of 256 keep the
// launch far below 2^32 threads at any state size.
static inline unsigned grid_for(uint64_t work, unsigned block) {
    const uint64_t b = (work + block - 1) / block;
    return (unsigned)(b > (1ull << 20) ? (1ull << 20) : b);
}

template <typename R, int K>
static hipError_t launch_dense_t(void *psi, uint64_t ngroups, const IndexArgs &ia,
                                 const DenseArgs &a, hipStream_t s) {
    constexpr int D = 1 << K;
    DenseArgsT<R, D> t;
    for (int i = 0; i < D * D; ++i) {
        t.mr[i] = (R)a.mr[i];
        t.mi[i] = (R)a.mi[i];
    }
    for (int i = 0; i < D; ++i) t.off[i] = a.off[i];
    if (ngroups == 0) return hipSuccess;
    hipLaunchKernelGGL((k_dense<R, K>), dim3(grid_for(ngroups, 256)), dim3(256), 0, s,
                       (typename V2<R>::T *)psi, ngroups, ia, t);
    return hipGetLastError();
}

hipError_t launch_dense(int dtype, void *psi, int k, uint64_t ngroups, const IndexArgs &ia,
                        const DenseArgs &a, hipStream_t s) {
    if (dtype == 0) {
        switch (k) {
        case 1: return launch_dense_t<double, 1>(psi, ngroups, ia, a, s);
        case 2: return launch_dense_t<double, 2>(psi, ngroups, ia, a, s);
        case 3: return launch_dense_t<double, 3>(psi, ngroups, ia, a, s);
        }
    } else {
        switch (k) {
        case 1: return launch_dense_t<float, 1>(psi, ngroups, ia, a, s);
        case 2: return launch_dense_t<float, 2>(psi, ngroups, ia, a, s);
        case 3: return launch_dense_t<float, 3>(psi, ngroups, ia, a, s);
        }
    }
    return hipErrorInvalidValue;
}

template <typename R, int K>
static hipError_t launch_mono_t(void *psi, uint64_t ngroups, const IndexArgs &ia,
                                const MonoArgs &a, hipStream_t s) {
    MonoArgsT<R> t;
    for (int i = 0; i < 32; ++i) {
        t.vr[i] = (R)a.vr[i];
        t.vi[i] = (R)a.vi[i];
        t.off[i] = a.off[i];
        t.srcoff[i] = a.srcoff[i];
    }
    t.touch = a.touch;
    if (ngroups == 0 || a.touch == 0) return hipSuccess;
    hipLaunchKernelGGL((k_mono<R, K>), dim3(grid_for(ngroups, 256)), dim3(256), 0, s,
                       (typename V2<R>::T *)psi, ngroups, ia, t);
    return hipGetLastError();
}

hipError_t launch_mono(int dtype, void *psi, int k, uint64_t ngroups, const IndexArgs &ia,
                       const MonoArgs &a, hipStream_t s) {
#define QSV_MONO_CASE(R)                                              \
    switch (k) {                                                      \
    case 1: return launch_mono_t<R, 1>(psi, ngroups, ia, a, s);       \
    case 2: return launch_mono_t<R, 2>(psi, ngroups, ia, a, s);       \
    case 3: return launch_mono_t<R, 3>(psi, ngroups, ia, a, s);       \
    case 4: return launch_mono_t<R, 4>(psi, ngroups, ia, a, s);       \
    case 5: return launch_mono_t<R, 5>(psi, ngroups, ia, a, s);       \
    }
    if (dtype == 0) {
        QSV_MONO_CASE(double)
    } else {
        QSV_MONO_CASE(float)
    }
#undef QSV_MONO_CASE
    return hipErrorInvalidValue;
}

}  // namespace dev
}  // namespace qsv
