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

// Amplitude loads and stores through global (address space 1) pointers.  A
// pointer that went through an empty asm, or a copy of the vector struct,
// loses the address space and compiles to flat accesses, which also count
// against the LDS wait counter: every LDS or scalar-load wait then waits for
// the tile's HBM traffic too.
typedef double __attribute__((ext_vector_type(2))) dvec2;
typedef float __attribute__((ext_vector_type(2))) fvec2;
typedef __attribute__((address_space(1))) dvec2 g_dvec2;
typedef __attribute__((address_space(1))) fvec2 g_fvec2;
__device__ __forceinline__ double2 gload(const double2 *p) {
    const dvec2 v = *(const g_dvec2 *)p;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 gload(const float2 *p) {
    const fvec2 v = *(const g_fvec2 *)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gstore(double2 *p, double2 a) {
    dvec2 v;
    v.x = a.x;
    v.y = a.y;
    *(g_dvec2 *)p = v;
}
__device__ __forceinline__ void gstore(float2 *p, float2 a) {
    fvec2 v;
    v.x = a.x;
    v.y = a.y;
    *(g_fvec2 *)p = v;
}

// LDS accesses at byte addresses formed as integers.  An access through a
// pointer into the dynamic LDS block compiles to an add of the block's base
// (a link-time symbol, 0 in a kernel without static LDS) before every access;
// an address formed once per op, base included, and XORed per access saves
// that add.  The XOR equals the add where the base is a multiple of the span
// of the XORed bits, which the callers check on the host (no static LDS: the
// dynamic block starts at 0).
typedef __attribute__((address_space(3))) dvec2 l_dvec2;
typedef __attribute__((address_space(3))) fvec2 l_fvec2;
typedef __attribute__((address_space(3))) uint32_t l_u32;
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}
__device__ __forceinline__ void lds_read(uint32_t a, double2 &out) {
    const dvec2 v = *(const l_dvec2 *)(uintptr_t)a;
    out = make_double2(v.x, v.y);
}
__device__ __forceinline__ void lds_read(uint32_t a, float2 &out) {
    const fvec2 v = *(const l_fvec2 *)(uintptr_t)a;
    out = make_float2(v.x, v.y);
}
__device__ __forceinline__ uint32_t lds_read_u32(uint32_t a) { return *(const l_u32 *)(uintptr_t)a; }
__device__ __forceinline__ void lds_write(uint32_t a, double2 x) {
    dvec2 v;
    v.x = x.x;
    v.y = x.y;
    *(l_dvec2 *)(uintptr_t)a = v;
}
__device__ __forceinline__ void lds_write(uint32_t a, float2 x) {
    fvec2 v;
    v.x = x.x;
    v.y = x.y;
    *(l_fvec2 *)(uintptr_t)a = v;
}

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

__device__ __forceinline__ uint64_t deposit_bits(uint32_t l, const uint32_t *tpos, int m) {
    uint64_t out = 0;
    for (int i = 0; i < m; ++i) out |= (uint64_t)((l >> i) & 1u) << tpos[i];
    return out;
}

// XOR of parts[b] over the set bits b of x (b < nbits, nbits <= 16).
__device__ __forceinline__ uint32_t xor_parts(uint32_t x, const uint32_t *parts, int nbits) {
    uint32_t o = 0;
    for (int b = 0; b < nbits; ++b) o ^= (0u - ((x >> b) & 1u)) & parts[b];
    return o;
}

// The same over N parts read once into registers (parts beyond nbits are
// zero), so a loop over x costs no memory reads.
template <int N> struct Parts {
    uint32_t v[N];
    __device__ __forceinline__ Parts(const uint32_t *parts, int nbits) {
#pragma unroll
        for (int b = 0; b < N; ++b) v[b] = b < nbits ? parts[b] : 0u;
    }
    __device__ __forceinline__ uint32_t of(uint32_t x) const {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) o ^= (0u - ((x >> b) & 1u)) & v[b];
        return o;
    }
};

// ----------------------------------------------------- ops on an LDS tile
// The tile is addressed in bytes through the op's precomputed offsets.
// Group g = threadIdx.x + kNT * it: the thread part of its address is fixed
// for the op, the iteration part is uniform.
// (Op fields and matrix entries are read into registers before the loops:
// inside them, the LDS stores would otherwise force the compiler to read
// them again on every iteration.)
template <typename R, int K>
__device__ __forceinline__ void lds_dense(unsigned char *tb, const TileOp &op,
                                          const typename VT<R>::T *__restrict__ mat) {
    using T = typename VT<R>::T;
    constexpr int D = 1 << K;
    const int nfree = op.nfree;
    const uint32_t ngroups = 1u << nfree;
    const uint32_t tid = threadIdx.x;
    const uint32_t toff = xor_parts(tid, op.fz, nfree < 8 ? nfree : 8);
    const Parts<8> hi(op.fz + 8, nfree - 8);
    uint32_t sl[D];
    T u[D * D];
#pragma unroll
    for (int r = 0; r < D; ++r) sl[r] = op.sl[r];
#pragma unroll
    for (int e = 0; e < D * D; ++e) u[e] = mat[e];
    for (uint32_t it = 0; it * kNT < ngroups; ++it) {
        if (tid >= ngroups) break;   // fewer groups than threads
        const uint32_t go = toff ^ hi.of(it);
        T x[D];
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = *reinterpret_cast<const T *>(tb + (go ^ sl[c]));
        // the whole group is in registers, so rows can be written one by one
#pragma unroll
        for (int r = 0; r < D; ++r) {
            T y = cmul(u[r * D], x[0]);
#pragma unroll
            for (int c = 1; c < D; ++c) y = cmadd(y, u[r * D + c], x[c]);
            *reinterpret_cast<T *>(tb + (go ^ sl[r])) = y;
        }
    }
}

template <typename R, int K>
__device__ __forceinline__ void lds_mono(unsigned char *tb, const TileOp &op,
                                         const typename VT<R>::T *__restrict__ val) {
    using T = typename VT<R>::T;
    constexpr int D = 1 << K;
    const int nfree = op.nfree;
    const uint32_t ngroups = 1u << nfree;
    const uint32_t tid = threadIdx.x;
    const uint32_t toff = xor_parts(tid, op.fz, nfree < 8 ? nfree : 8);
    const Parts<8> hi(op.fz + 8, nfree - 8);
    // untouched rows read and write their own amplitude with phase 1
    uint32_t sl[D], ss[D];
    T v[D];
    const uint32_t touch = op.touch;
#pragma unroll
    for (int r = 0; r < D; ++r) {
        const bool t = (touch >> r) & 1;
        sl[r] = op.sl[r];
        ss[r] = t ? op.ss[r] : sl[r];
        T one;
        one.x = R(1);
        one.y = R(0);
        v[r] = t ? val[r] : one;
    }
    for (uint32_t it = 0; it * kNT < ngroups; ++it) {
        if (tid >= ngroups) break;
        const uint32_t go = toff ^ hi.of(it);
        T y[D];
#pragma unroll
        for (int r = 0; r < D; ++r)
            y[r] = cmul(v[r], *reinterpret_cast<const T *>(tb + (go ^ ss[r])));
#pragma unroll
        for (int r = 0; r < D; ++r) *reinterpret_cast<T *>(tb + (go ^ sl[r])) = y[r];
    }
}

// ------------------------------------------------------ matrix-core ops
// A dense k-qubit op (k = 3..5) on the tile as a real GEMM Y = W X on the
// 16x16x4 MFMA: X holds one group of 2^k amplitudes per column as
// [Re x; Im x] (2^(k+1) rows), W is the real embedding of U.  A wave takes 16
// groups at a time (one B column per lane % 16, lane bits 0..3 = free bits
// 0..3 of the group).  The host stores W in fragment order, so the A operand
// of each MFMA is one contiguous, cache-resident read across the wave.
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
__device__ __forceinline__ void lds_dense_mfma(unsigned char *tb, const TileOp &op,
                                               const R *__restrict__ W) {
    using V = typename Mfma<R>::V;
    constexpr int D = 1 << K, D2 = 2 * D;
    constexpr int MB = D2 / 16, KC = D2 / 4;
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nwaves = blockDim.x >> 6;
    const int nfree = op.nfree;
    const uint32_t ngroups = 1u << nfree;
    const uint32_t ncb = (ngroups + 15) >> 4;
    const uint32_t loff = xor_parts((uint32_t)lane & 15u, op.fz, nfree < 4 ? nfree : 4);
    const bool valid = ((uint32_t)lane & 15u) < ngroups;
    // the lane's row offsets (read once per op, kept in registers)
    uint32_t in_off[KC], out_off[MB][4];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        const int rho = 4 * kc + (lane >> 4);
        in_off[kc] = op.sl[rho & (D - 1)] | (rho >= D ? (uint32_t)sizeof(R) : 0u);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * mb + Mfma<R>::row(lane, r);
            out_off[mb][r] = op.sl[row & (D - 1)] | (row >= D ? (uint32_t)sizeof(R) : 0u);
        }
    const R *wl = W + lane;
    const Parts<12> hi(op.fz + 4, nfree - 4);
    for (uint32_t cb = wave; cb < ncb; cb += nwaves) {
        const uint32_t go = loff ^ hi.of(cb);
        V acc[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = V{0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const R b = valid ? *reinterpret_cast<const R *>(tb + (go ^ in_off[kc])) : R(0);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                acc[mb] = Mfma<R>::op(wl[(mb * KC + kc) * 64], b, acc[mb]);
        }
        if (valid) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    *reinterpret_cast<R *>(tb + (go ^ out_off[mb][r])) = acc[mb][r];
        }
    }
}

// Apply LDS op `op` to the whole tile (all threads take part).  KM is the
// widest matrix-core op the caller can meet (0: none); the host emits dense
// ops of 3 or more qubits only in matrix-core form.
template <typename R, int KM = 5>
__device__ void lds_op(typename VT<R>::T *tile, int m, uint64_t base, const uint32_t *tpos,
                       const TileOp &op, const typename VT<R>::T *__restrict__ pool,
                       const uint64_t *dep_hi = nullptr) {
    using T = typename VT<R>::T;
    if ((base & op.ectrl) != op.ectrl) return;
    const T *mat = pool + op.mat;
    unsigned char *tb = reinterpret_cast<unsigned char *>(tile);
    if (op.kind == TOP_DENSE_MFMA) {
        const R *W = reinterpret_cast<const R *>(mat);
        if constexpr (KM >= 3) {
            if (op.k == 3) lds_dense_mfma<R, 3>(tb, op, W);
        }
        if constexpr (KM >= 4) {
            if (op.k == 4) lds_dense_mfma<R, 4>(tb, op, W);
        }
        if constexpr (KM >= 5) {
            if (op.k == 5) lds_dense_mfma<R, 5>(tb, op, W);
        }
    } else if (op.kind == TOP_DENSE) {
        if (op.k == 1) lds_dense<R, 1>(tb, op, mat);
        else lds_dense<R, 2>(tb, op, mat);
    } else if (op.kind == TOP_MONO) {
        // (the host lowers monomial ops of 4 or more qubits as dense ops)
        if (op.k == 1) lds_mono<R, 1>(tb, op, mat);
        else if (op.k == 2) lds_mono<R, 2>(tb, op, mat);
        else lds_mono<R, 3>(tb, op, mat);
    } else {
        // diagonal op with targets outside the tile: the phase index and the
        // controls come from the global index of each amplitude
        const uint32_t tsize = 1u << m;
        const uint32_t tid = threadIdx.x;
        const uint64_t dep_tid = deposit_bits(tid & (tsize - 1), tpos, m);
        for (uint32_t j = 0; j < tsize; j += kNT) {
            const uint32_t l = j + tid;
            if (l >= tsize) break;
            const uint64_t gi =
                base | dep_tid | (dep_hi ? dep_hi[j >> 8] : deposit_bits(j, tpos, m));
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
