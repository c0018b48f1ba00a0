// Gate kernels for gfx950: per-gate dense and monomial updates streaming the
// state through HBM, and the LDS-tile pass that applies a list of operations
// to 2^m-amplitude tiles with one HBM read and one HBM write per amplitude.
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
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
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

template <typename R, int K>
__global__ __launch_bounds__(256) void k_mono(typename V2<R>::T *__restrict__ psi,
                                              uint64_t ngroups, IndexArgs ia, MonoArgsT<R> a) {
    using T = typename V2<R>::T;
    constexpr int D = 1 << K;
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups) return;
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

static inline unsigned grid_for(uint64_t work, unsigned block) {
    return (unsigned)((work + block - 1) / block);
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

// --------------------------------------------------------------- tile pass
constexpr int kTileThreads = 256;

__device__ __forceinline__ uint32_t insert_local(uint32_t g, const uint8_t *pos, int npos) {
    for (int i = 0; i < npos; ++i) {
        const uint32_t lowm = (1u << pos[i]) - 1;
        g = ((g & ~lowm) << 1) | (g & lowm);
    }
    return g;
}

template <typename R, int K>
__device__ __forceinline__ void tile_dense(typename V2<R>::T *tile, int m, const TileOp &op,
                                           const typename V2<R>::T *__restrict__ mat) {
    using T = typename V2<R>::T;
    constexpr int D = 1 << K;
    const int npos = op.npos;
    const uint32_t ngroups = 1u << (m - npos);
    const uint32_t lctrl = op.lctrl;
    for (uint32_t g = threadIdx.x; g < ngroups; g += kTileThreads) {
        const uint32_t l0 = insert_local(g, op.pos, npos) | lctrl;
        T x[D];
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = tile[l0 + op.loff[c]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            R yr = 0, yi = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const T u = mat[r * D + c];
                yr += u.x * x[c].x - u.y * x[c].y;
                yi += u.x * x[c].y + u.y * x[c].x;
            }
            T y;
            y.x = yr;
            y.y = yi;
            tile[l0 + op.loff[r]] = y;
        }
    }
}

template <typename R, int K>
__device__ __forceinline__ void tile_mono(typename V2<R>::T *tile, int m, const TileOp &op,
                                          const typename V2<R>::T *__restrict__ val) {
    using T = typename V2<R>::T;
    constexpr int D = 1 << K;
    const int npos = op.npos;
    const uint32_t ngroups = 1u << (m - npos);
    const uint32_t lctrl = op.lctrl, touch = op.touch;
    for (uint32_t g = threadIdx.x; g < ngroups; g += kTileThreads) {
        const uint32_t l0 = insert_local(g, op.pos, npos) | lctrl;
        T y[D];
#pragma unroll
        for (int r = 0; r < D; ++r)
            if ((touch >> r) & 1) {
                const T s = tile[l0 + op.srcoff[r]];
                const T v = val[r];
                y[r].x = v.x * s.x - v.y * s.y;
                y[r].y = v.x * s.y + v.y * s.x;
            }
#pragma unroll
        for (int r = 0; r < D; ++r)
            if ((touch >> r) & 1) tile[l0 + op.loff[r]] = y[r];
    }
}

__device__ __forceinline__ uint64_t deposit(uint32_t l, const uint8_t *tpos, int m) {
    uint64_t out = 0;
    for (int i = 0; i < m; ++i) out |= (uint64_t)((l >> i) & 1u) << tpos[i];
    return out;
}

template <typename R>
__global__ __launch_bounds__(kTileThreads) void k_tile(typename V2<R>::T *__restrict__ psi,
                                                       TileArgs ta,
                                                       const TileOp *__restrict__ ops,
                                                       const typename V2<R>::T *__restrict__ pool) {
    using T = typename V2<R>::T;
    extern __shared__ unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);
    const int m = ta.m;
    const uint32_t tsize = 1u << m;
    // Base index of the tile: the block id with zeros inserted at the tile bits.
    uint64_t base = (uint64_t)blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
    for (int i = 0; i < m; ++i) {
        const uint64_t lowm = (1ull << ta.tpos[i]) - 1;
        base = ((base & ~lowm) << 1) | (base & lowm);
    }
    const uint32_t tid = threadIdx.x;
    // deposit(l) = deposit(tid) | deposit(l - tid) for l = tid + j*256
    const uint64_t dep_tid = deposit(tid & (tsize - 1), ta.tpos, m);
    for (uint32_t j = 0; j < tsize; j += kTileThreads) {
        const uint32_t l = j + tid;
        if (l < tsize) tile[l] = psi[base | dep_tid | deposit(j, ta.tpos, m)];
    }
    __syncthreads();
    for (int oi = 0; oi < ta.n_ops; ++oi) {
        const TileOp &op = ops[oi];
        if ((base & op.ectrl) != op.ectrl) continue;   // uniform over the block
        const T *mat = pool + op.mat;
        if (op.kind == TOP_DENSE) {
            switch (op.k) {
            case 1: tile_dense<R, 1>(tile, m, op, mat); break;
            case 2: tile_dense<R, 2>(tile, m, op, mat); break;
            case 3: tile_dense<R, 3>(tile, m, op, mat); break;
            case 4: tile_dense<R, 4>(tile, m, op, mat); break;
            case 5: tile_dense<R, 5>(tile, m, op, mat); break;
            }
        } else if (op.kind == TOP_MONO) {
            switch (op.k) {
            case 1: tile_mono<R, 1>(tile, m, op, mat); break;
            case 2: tile_mono<R, 2>(tile, m, op, mat); break;
            case 3: tile_mono<R, 3>(tile, m, op, mat); break;
            case 4: tile_mono<R, 4>(tile, m, op, mat); break;
            case 5: tile_mono<R, 5>(tile, m, op, mat); break;
            }
        } else {
            // diagonal with targets anywhere: entry from the global index
            const int k = op.k;
            const uint64_t gctrl = op.gctrl;
            const uint32_t touch = op.touch;
            for (uint32_t j = 0; j < tsize; j += kTileThreads) {
                const uint32_t l = j + tid;
                if (l >= tsize) break;
                const uint64_t gi = base | dep_tid | deposit(j, ta.tpos, m);
                if ((gi & gctrl) != gctrl) continue;
                uint32_t r = 0;
                for (int q = 0; q < k; ++q) r |= (uint32_t)((gi >> op.gt[q]) & 1u) << q;
                if (!((touch >> r) & 1)) continue;
                const T v = mat[r];
                const T s = tile[l];
                T y;
                y.x = v.x * s.x - v.y * s.y;
                y.y = v.x * s.y + v.y * s.x;
                tile[l] = y;
            }
        }
        __syncthreads();
    }
    for (uint32_t j = 0; j < tsize; j += kTileThreads) {
        const uint32_t l = j + tid;
        if (l < tsize) psi[base | dep_tid | deposit(j, ta.tpos, m)] = tile[l];
    }
}

int tile_pass_max_bits(int dtype) { return dtype == 0 ? 13 : 14; }

template <typename R>
static hipError_t launch_tile_t(void *psi, const TileArgs &ta, const TileOp *ops,
                                const void *pool, hipStream_t s) {
    using T = typename V2<R>::T;
    const size_t lds = (size_t)sizeof(T) << ta.m;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_tile<R>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(sizeof(T) << tile_pass_max_bits(sizeof(R) == 8 ? 0 : 1)));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    uint64_t nt = ta.n_tiles;
    if (nt == 0) return hipSuccess;
    dim3 grid;
    if (nt <= 0x7fffffffull) {
        grid = dim3((unsigned)nt, 1, 1);
    } else {
        grid = dim3(1u << 30, (unsigned)(nt >> 30), 1);
    }
    hipLaunchKernelGGL((k_tile<R>), grid, dim3(kTileThreads), lds, s, (T *)psi, ta, ops,
                       (const T *)pool);
    return hipGetLastError();
}

hipError_t launch_tile_pass(int dtype, void *psi, const TileArgs &ta, const TileOp *ops,
                            const void *pool, hipStream_t s) {
    if (ta.m < 1 || ta.m > tile_pass_max_bits(dtype)) return hipErrorInvalidValue;
    return dtype == 0 ? launch_tile_t<double>(psi, ta, ops, pool, s)
                      : launch_tile_t<float>(psi, ta, ops, pool, s);
}

}  // namespace dev
}  // namespace qsv
