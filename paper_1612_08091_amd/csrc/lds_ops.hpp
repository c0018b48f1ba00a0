// Device helpers shared by the tile kernels and the batched kernel: complex
// arithmetic, the LDS index swizzle and the operations that sweep a tile
// held in LDS (dense, monomial and diagonal-on-global-bits updates).
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace qsv {
namespace dev {

template <typename R> struct VT;
template <> struct VT<double> { using T = double2; };
template <> struct VT<float> { using T = float2; };

// XOR swizzle of an LDS element index: the bits above the 256-byte bank span
// are folded into the bits below it.  A bijection on [0, 2^m).
template <typename R> __device__ __forceinline__ uint32_t swz(uint32_t l);
template <> __device__ __forceinline__ uint32_t swz<double>(uint32_t l) {
    return l ^ (((l >> 4) ^ (l >> 8)) & 15u);
}
template <> __device__ __forceinline__ uint32_t swz<float>(uint32_t l) {
    return l ^ (((l >> 5) ^ (l >> 10)) & 31u);
}

template <typename T> __device__ __forceinline__ T cmul(const T &a, const T &b) {
    T r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename T> __device__ __forceinline__ T cmadd(const T &acc, const T &a, const T &b) {
    T r;
    r.x = acc.x + a.x * b.x - a.y * b.y;
    r.y = acc.y + a.x * b.y + a.y * b.x;
    return r;
}
template <typename T> __device__ __forceinline__ T csel(bool c, const T &a, const T &b) {
    T r;
    r.x = c ? a.x : b.x;
    r.y = c ? a.y : b.y;
    return r;
}

constexpr int kNT = 256;

__device__ __forceinline__ uint32_t insert_local(uint32_t g, const uint8_t *pos, int npos) {
    for (int i = 0; i < npos; ++i) {
        const uint32_t lowm = (1u << pos[i]) - 1;
        g = ((g & ~lowm) << 1) | (g & lowm);
    }
    return g;
}

// ----------------------------------------------------- ops on an LDS tile
// The tile is addressed through swz(); l is the logical local index.
template <typename R, int K>
__device__ __forceinline__ void lds_dense(typename VT<R>::T *tile, int m, const TileOp &op,
                                          const typename VT<R>::T *__restrict__ mat) {
    using T = typename VT<R>::T;
    constexpr int D = 1 << K;
    const int npos = op.npos;
    const uint32_t ngroups = 1u << (m - npos);
    const uint32_t lctrl = op.lctrl;
    for (uint32_t g = threadIdx.x; g < ngroups; g += kNT) {
        const uint32_t l0 = insert_local(g, op.pos, npos) | lctrl;
        T x[D];
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = tile[swz<R>(l0 + op.loff[c])];
        // the whole group is in registers, so rows can be written one by one
        if constexpr (K <= 3) {
#pragma unroll
            for (int r = 0; r < D; ++r) {
                T y;
                y.x = 0;
                y.y = 0;
#pragma unroll
                for (int c = 0; c < D; ++c) y = cmadd(y, mat[r * D + c], x[c]);
                tile[swz<R>(l0 + op.loff[r])] = y;
            }
        } else {
#pragma unroll 1
            for (int r = 0; r < D; ++r) {
                T y;
                y.x = 0;
                y.y = 0;
#pragma unroll
                for (int c = 0; c < D; ++c) y = cmadd(y, mat[r * D + c], x[c]);
                tile[swz<R>(l0 + op.loff[r])] = y;
            }
        }
    }
}

template <typename R, int K>
__device__ __forceinline__ void lds_mono(typename VT<R>::T *tile, int m, const TileOp &op,
                                         const typename VT<R>::T *__restrict__ val) {
    using T = typename VT<R>::T;
    constexpr int D = 1 << K;
    const int npos = op.npos;
    const uint32_t ngroups = 1u << (m - npos);
    const uint32_t lctrl = op.lctrl, touch = op.touch;
    for (uint32_t g = threadIdx.x; g < ngroups; g += kNT) {
        const uint32_t l0 = insert_local(g, op.pos, npos) | lctrl;
        T y[D];
#pragma unroll
        for (int r = 0; r < D; ++r)
            if ((touch >> r) & 1) y[r] = cmul(val[r], tile[swz<R>(l0 + op.srcoff[r])]);
#pragma unroll
        for (int r = 0; r < D; ++r)
            if ((touch >> r) & 1) tile[swz<R>(l0 + op.loff[r])] = y[r];
    }
}

__device__ __forceinline__ uint64_t deposit_bits(uint32_t l, const uint8_t *tpos, int m) {
    uint64_t out = 0;
    for (int i = 0; i < m; ++i) out |= (uint64_t)((l >> i) & 1u) << tpos[i];
    return out;
}

// Apply LDS op `op` to the whole tile (all threads take part).
template <typename R>
__device__ void lds_op(typename VT<R>::T *tile, int m, uint64_t base, const TileArgs &ta,
                       const TileOp &op, const typename VT<R>::T *__restrict__ pool) {
    using T = typename VT<R>::T;
    if ((base & op.ectrl) != op.ectrl) return;
    const T *mat = pool + op.mat;
    if (op.kind == TOP_DENSE) {
        switch (op.k) {
        case 1: lds_dense<R, 1>(tile, m, op, mat); break;
        case 2: lds_dense<R, 2>(tile, m, op, mat); break;
        case 3: lds_dense<R, 3>(tile, m, op, mat); break;
        case 4: lds_dense<R, 4>(tile, m, op, mat); break;
        case 5: lds_dense<R, 5>(tile, m, op, mat); break;
        }
    } else if (op.kind == TOP_MONO) {
        switch (op.k) {
        case 1: lds_mono<R, 1>(tile, m, op, mat); break;
        case 2: lds_mono<R, 2>(tile, m, op, mat); break;
        case 3: lds_mono<R, 3>(tile, m, op, mat); break;
        case 4: lds_mono<R, 4>(tile, m, op, mat); break;
        case 5: lds_mono<R, 5>(tile, m, op, mat); break;
        }
    } else {
        const uint32_t tsize = 1u << m;
        for (uint32_t l = threadIdx.x; l < tsize; l += kNT) {
            const uint64_t gi = base | deposit_bits(l, ta.tpos, m);
            if ((gi & op.gctrl) != op.gctrl) continue;
            uint32_t r = 0;
            for (int q = 0; q < op.k; ++q) r |= (uint32_t)((gi >> op.gt[q]) & 1u) << q;
            if (!((op.touch >> r) & 1)) continue;
            const uint32_t p = swz<R>(l);
            tile[p] = cmul(mat[r], tile[p]);
        }
    }
}

}  // namespace dev
}  // namespace qsv
