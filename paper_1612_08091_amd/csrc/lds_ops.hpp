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

// ------------------------------------------------------ matrix-core ops
// A dense k-qubit op (k = 3..5) on the tile as a real GEMM Y = W X on the
// 16x16x4 MFMA: X holds one group of 2^k amplitudes per column as
// [Re x; Im x] (2^(k+1) rows), W is the real embedding of U.  A wave takes 16
// groups at a time (one B column per lane % 16); the W fragments a lane
// feeds to the A operand stay in registers for the whole op.
typedef float qsv_v4f __attribute__((ext_vector_type(4)));
typedef double qsv_v4d __attribute__((ext_vector_type(4)));

template <typename R> struct Mfma;
template <> struct Mfma<float> {
    using V = qsv_v4f;
    static __device__ __forceinline__ V op(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // row of the 16x16 result held in accumulator element r of lane l
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct Mfma<double> {
    using V = qsv_v4d;
    static __device__ __forceinline__ V op(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};

template <typename R, int K>
__device__ __forceinline__ void lds_dense_mfma(typename VT<R>::T *tile, int m, const TileOp &op,
                                               const R *__restrict__ W) {
    using V = typename Mfma<R>::V;
    constexpr int D = 1 << K, D2 = 2 * D;
    constexpr int MB = D2 / 16, KC = D2 / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int npos = op.npos;
    const uint32_t ngroups = 1u << (m - npos);
    const uint32_t ncb = (ngroups + 15) >> 4;
    R a[MB][KC];
    uint32_t in_off[KC];
    int in_part[KC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        const int rho = 4 * kc + (lane >> 4);
        in_off[kc] = op.loff[rho & (D - 1)];
        in_part[kc] = rho >= D;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) a[mb][kc] = W[(16 * mb + (lane & 15)) * D2 + rho];
    }
    uint32_t out_off[MB][4];
    int out_part[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * mb + Mfma<R>::row(lane, r);
            out_off[mb][r] = op.loff[row & (D - 1)];
            out_part[mb][r] = row >= D;
        }
    R *tr = reinterpret_cast<R *>(tile);
    for (uint32_t cb = wave; cb < ncb; cb += nwaves) {
        const uint32_t g = cb * 16 + (lane & 15);
        const bool valid = g < ngroups;
        const uint32_t l0 = valid ? (insert_local(g, op.pos, npos) | op.lctrl) : 0u;
        V acc[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = V{0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const R b = valid ? tr[2 * swz<R>(l0 + in_off[kc]) + in_part[kc]] : R(0);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = Mfma<R>::op(a[mb][kc], b, acc[mb]);
        }
        if (valid) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    tr[2 * swz<R>(l0 + out_off[mb][r]) + out_part[mb][r]] = acc[mb][r];
        }
    }
}

// Apply LDS op `op` to the whole tile (all threads take part).
template <typename R>
__device__ void lds_op(typename VT<R>::T *tile, int m, uint64_t base, const TileArgs &ta,
                       const TileOp &op, const typename VT<R>::T *__restrict__ pool) {
    using T = typename VT<R>::T;
    if ((base & op.ectrl) != op.ectrl) return;
    const T *mat = pool + op.mat;
    if (op.kind == TOP_DENSE_MFMA) {
        const R *W = reinterpret_cast<const R *>(mat);
        switch (op.k) {
        case 3: lds_dense_mfma<R, 3>(tile, m, op, W); break;
        case 4: lds_dense_mfma<R, 4>(tile, m, op, W); break;
        case 5: lds_dense_mfma<R, 5>(tile, m, op, W); break;
        }
    } else if (op.kind == TOP_DENSE) {
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
