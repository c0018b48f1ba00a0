// LDS-tile passes for gfx950.  One workgroup owns a tile: the 2^m amplitudes
// whose indices agree outside the m tile bits.  The tile is read from HBM
// once, every operation of the pass is applied to it on chip, and it is
// written back once, so a pass costs one read and one write of the state
// whatever the number of gates it holds (the lazily cached gates of Sec.
// 4.3.2 executed in bulk).
//
// Two kernels:
//  * k_tile_reg<R, RB, TB>: m = RB + TB.  Each of the 2^TB threads keeps
//    2^RB amplitudes in registers.  Register bit j and thread bit i each
//    stand for one tile bit (the layout).  1- and 2-qubit operations on
//    register bits run in registers, as complex matrices or, when the host
//    split them into phases times a real matrix, as real matrices at half the
//    arithmetic; diagonal operations multiply by factors from tables that the
//    workgroup keeps in LDS; a REMAP op moves the tile through LDS (XOR
//    swizzled against bank conflicts) into a new layout.  Every
//    layout-dependent offset comes precomputed from the host.  Passes holding
//    wider operations use k_tile_lds.
//  * k_tile_lds<R>: any m <= 14; the tile lives in LDS and every operation
//    sweeps it (used for small states).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "lds_ops.hpp"

namespace qsv {
namespace dev {

// ------------------------------------------------------- k_tile_lds
// Persistent like k_tile_reg: resident workgroups take tiles from a per-pass
// counter that the host zeroes.
template <typename R, int KM>
__global__ __launch_bounds__(kNT) void k_tile_lds(typename VT<R>::T *__restrict__ psi,
                                                  TileArgs ta, const TileOp *__restrict__ ops,
                                                  const typename VT<R>::T *__restrict__ pool,
                                                  unsigned int *__restrict__ counter) {
    using T = typename VT<R>::T;
    // the tile at the start of dynamic LDS (address 0), the tile counter's
    // broadcast slot right after it
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);
    unsigned int &s_tile = *reinterpret_cast<unsigned int *>(smem_raw + (sizeof(T) << ta.m));
    const int m = ta.m;
    const uint32_t tsize = 1u << m;
    const uint32_t tid = threadIdx.x;
    // this thread's share of every tile: local indices j + tid, j = 0, kNT, ...
    const uint64_t dep_tid = deposit_bits(tid & (tsize - 1), ta.tpos, m);
    const uint64_t dep_tid_f = deposit_bits(tid & (tsize - 1), ta.spos, m);
    const uint32_t swz_tid = swz<R>(tid & (tsize - 1));
    const uint32_t n_tiles = (uint32_t)ta.n_tiles;
    if (tid == 0) s_tile = atomicAdd(counter, 1u);
    __syncthreads();
    uint32_t t = __builtin_amdgcn_readfirstlane(s_tile);
    while (t < n_tiles) {
        uint64_t base = t;
        for (int i = 0; i < m; ++i) {
            const uint64_t lowm = (1ull << ta.tpos[i]) - 1;
            base = ((base & ~lowm) << 1) | (base & lowm);
        }
        // loads in batches of 8 per thread, all in flight before their LDS
        // writes (one HBM round trip per batch, not per amplitude)
        if (tsize >= 8 * kNT) {
            for (uint32_t j0 = 0; j0 < tsize; j0 += 8 * kNT) {
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    v[u] = gload(psi + (base | dep_tid | ta.dep_hi[(j0 >> 8) + u]));
#pragma unroll
                for (int u = 0; u < 8; ++u) tile[swz_tid ^ swz<R>(j0 + u * kNT)] = v[u];
            }
        } else {
            for (uint32_t j = 0; j < tsize; j += kNT)
                if (j + tid < tsize)
                    tile[swz_tid ^ swz<R>(j)] = gload(psi + (base | dep_tid | ta.dep_hi[j >> 8]));
        }
        unsigned int next = 0;
        if (tid == 0) next = atomicAdd(counter, 1u);
        // normal priority for the ops; raised again for the stores and the
        // next tile's loads (see k_tile_reg)
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        for (int oi = 0; oi < ta.n_ops; ++oi) {
            lds_op<R, KM>(tile, m, base, ta.tpos, ops[oi], pool, ta.dep_hi);
            __syncthreads();
        }
        __builtin_amdgcn_s_setprio(2);
        if (tsize >= 8 * kNT) {
            for (uint32_t j0 = 0; j0 < tsize; j0 += 8 * kNT) {
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = tile[swz_tid ^ swz<R>(j0 + u * kNT)];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    gstore(psi + (base | dep_tid_f | ta.dep_hi_f[(j0 >> 8) + u]), v[u]);
            }
        } else {
            for (uint32_t j = 0; j < tsize; j += kNT)
                if (j + tid < tsize)
                    gstore(psi + (base | dep_tid_f | ta.dep_hi_f[j >> 8]), tile[swz_tid ^ swz<R>(j)]);
        }
        if (tid == 0) s_tile = next;
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_tile);
    }
}

// ------------------------------------------------------- k_tile_reg
__device__ __forceinline__ double rfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float rfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Register ops run in place, one group of 2 or 4 amplitudes at a time, and
// never skip: an op under controls (CTRL) computes every group and keeps the
// old value where the controls fail, so the register allocation of the
// uncontrolled path holds no copies for a skipped case.  `on` is the lane's
// share of the controls (thread-id bits, bits outside the tile); creg holds
// the register bits that are controls.  Matrices arrive in scalar registers
// (m: the op's inline coefficients, row-major; complex ones as re, im).
template <typename T, typename R, int NR, int J, bool CTRL>
__device__ __forceinline__ void reg_g1(T *amp, const R *m, bool on, uint32_t creg) {
    T u[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        u[e].x = m[2 * e];
        u[e].y = m[2 * e + 1];
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & (1 << J)) continue;
        const int i1 = i | (1 << J);
        const T a = amp[i], b = amp[i1];
        T na = cmul(u[0], a);
        na = cmadd(na, u[1], b);
        T nb = cmul(u[2], a);
        nb = cmadd(nb, u[3], b);
        if (CTRL) {
            const bool c = on && ((i & creg) == creg);
            na = csel(c, na, a);
            nb = csel(c, nb, b);
        }
        amp[i] = na;
        amp[i1] = nb;
    }
}

template <typename T, typename R, int NR, int J1, int J2, bool CTRL>
__device__ __forceinline__ void reg_g2(T *amp, const R *m, bool on, uint32_t creg) {
    T u[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        u[e].x = m[2 * e];
        u[e].y = m[2 * e + 1];
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & ((1 << J1) | (1 << J2))) continue;
        const int idx[4] = {i, i | (1 << J1), i | (1 << J2), i | (1 << J1) | (1 << J2)};
        T x[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = amp[idx[c]];
        const bool c = !CTRL || (on && ((i & creg) == creg));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T y = cmul(u[r * 4], x[0]);
#pragma unroll
            for (int cc = 1; cc < 4; ++cc) y = cmadd(y, u[r * 4 + cc], x[cc]);
            amp[idx[r]] = CTRL ? csel(c, y, x[r]) : y;
        }
    }
}

// Real matrices: the real and imaginary parts of the amplitudes transform
// separately, 2 (1-qubit) or 4 (2-qubit) multiply-adds per part.
template <typename T, typename R, int NR, int J, bool CTRL>
__device__ __forceinline__ void reg_r1(T *amp, const R *m, bool on, uint32_t creg) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & (1 << J)) continue;
        const int i1 = i | (1 << J);
        const T a = amp[i], b = amp[i1];
        T na, nb;
        na.x = rfma(m[1], b.x, m[0] * a.x);
        na.y = rfma(m[1], b.y, m[0] * a.y);
        nb.x = rfma(m[3], b.x, m[2] * a.x);
        nb.y = rfma(m[3], b.y, m[2] * a.y);
        if (CTRL) {
            const bool c = on && ((i & creg) == creg);
            na = csel(c, na, a);
            nb = csel(c, nb, b);
        }
        amp[i] = na;
        amp[i1] = nb;
    }
}

template <typename T, typename R, int NR, int J1, int J2, bool CTRL>
__device__ __forceinline__ void reg_r2(T *amp, const R *m, bool on, uint32_t creg) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & ((1 << J1) | (1 << J2))) continue;
        const int idx[4] = {i, i | (1 << J1), i | (1 << J2), i | (1 << J1) | (1 << J2)};
        T x[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = amp[idx[c]];
        const bool c = !CTRL || (on && ((i & creg) == creg));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T y;
            y.x = m[r * 4] * x[0].x;
            y.y = m[r * 4] * x[0].y;
#pragma unroll
            for (int cc = 1; cc < 4; ++cc) {
                y.x = rfma(m[r * 4 + cc], x[cc].x, y.x);
                y.y = rfma(m[r * 4 + cc], x[cc].y, y.y);
            }
            amp[idx[r]] = CTRL ? csel(c, y, x[r]) : y;
        }
    }
}

// Diagonal op: amplitude i of the thread takes the factor at byte offset
// (lane part ^ wave part ^ tile part ^ wr[i]) of the op's table in the LDS
// image; the lane part places the lane's table bits (a bit-field extract and
// a shift per lane bit).  The four parts come from disjoint table bits (lane
// and wave thread-id bits, bits outside the tile, register bits), so the XOR
// is their sum; the table sits at a multiple of its size, so the offset
// never leaves it.  Controls inside the tile are table bits; a tile that
// fails the controls outside it reads a table of ones (at byte offset b)
// rather than skipping the op.  The reads go out four at a time.
template <typename T, int NR>
__device__ __forceinline__ void reg_diag(T *amp, const RegOp &op, uint32_t limg_a,
                                         uint64_t base, uint32_t lane, uint32_t wave) {
    uint32_t wr[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) wr[i] = op.wr[i];
    uint32_t sh[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) sh[t] = op.rd[t];
    const uint64_t lmask = op.lane_ok;
    uint32_t s_idx = (uint32_t)op.mat;
    if ((base & op.octrl) != op.octrl) s_idx = (uint32_t)op.b;
    s_idx ^= op.wwave[wave];
    for (int q = 0; q < op.a; ++q)
        if ((base >> op.gt[q]) & 1) s_idx ^= op.gtb[q];
    // the image's LDS address (a multiple of every table's size) joins the
    // uniform part; the lane and register parts then still OR and XOR in
    uint32_t v_idx = s_idx + limg_a;
    if (lmask != 0) {   // uniform: tables without lane bits skip the lane part
#pragma unroll
        for (int t = 0; t < 6; ++t)
            v_idx |= __builtin_amdgcn_ubfe(lane, (uint32_t)t, (uint32_t)((lmask >> t) & 1u)) << sh[t];
    }
#pragma unroll
    for (int i0 = 0; i0 < NR; i0 += 4) {
        T f[4];
#pragma unroll
        for (int i = 0; i < 4 && i0 + i < NR; ++i) lds_read(v_idx ^ wr[i0 + i], f[i]);
#pragma unroll
        for (int i = 0; i < 4 && i0 + i < NR; ++i) amp[i0 + i] = cmul(f[i], amp[i0 + i]);
    }
}

// Layout change through an LDS buffer of half a tile.  Slot J holds the same
// tile bit before and after, and the buffer drops that bit from the index.
// In phase p every thread writes its registers whose slot-J bit is p, then
// reads the same register indices in the new layout, so no register is
// overwritten before it was written out.  Addresses are the thread part XOR
// the (uniform) register part, both precomputed on the host; the register
// parts come in scalar registers, loaded before the first barrier.
// Ordering of LDS accesses within one wave: the wave's LDS operations run in
// order, so only the compiler has to be kept from moving them across.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// mode 1: a wave-local remap (each wave on its own region of the buffer, no
// workgroup barrier); 0: a workgroup remap; 2: a workgroup remap that first
// waits for every wave to leave its region of an earlier wave-local one.
template <typename T, int NR, int J>
__device__ __forceinline__ void remap_half(T *amp, uint32_t wt, uint32_t rt,
                                           const uint32_t *wr, const uint32_t *rd, int mode) {
    if (mode == 2) __syncthreads();
    // the thread parts pass through an empty asm in each phase, so the
    // addresses are formed next to their accesses (not all hoisted above the
    // barriers, which would hold 2^RB more VGPRs)
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        uint32_t w = wt;
        asm volatile("" : "+v"(w));
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (((i >> J) & 1) != p) continue;
            lds_write(w ^ wr[i], amp[i]);
        }
        if (mode == 1) wave_sync();
        else __syncthreads();
        uint32_t r = rt;
        asm volatile("" : "+v"(r));
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (((i >> J) & 1) != p) continue;
            lds_read(r ^ rd[i], amp[i]);
        }
        if (mode == 1) wave_sync();
        else __syncthreads();
    }
}

template <typename R> __device__ __forceinline__ const R *op_mat(const RegOp &op);
template <> __device__ __forceinline__ const double *op_mat<double>(const RegOp &op) { return op.md; }
template <> __device__ __forceinline__ const float *op_mat<float>(const RegOp &op) { return op.mf; }

#define QSV_SLOT1(J, CALL)                                        \
    case J:                                                       \
        if constexpr (RB > J) { CALL; } else __builtin_unreachable(); \
        break;

template <typename T, typename R, int NR, int RB, bool CTRL>
__device__ __forceinline__ void dispatch_1(T *amp, int kind, int j, const R *m, bool on,
                                           uint32_t creg) {
    if (kind == ROP_R1) {
        switch (j) {
            QSV_SLOT1(0, (reg_r1<T, R, NR, 0, CTRL>(amp, m, on, creg)))
            QSV_SLOT1(1, (reg_r1<T, R, NR, 1, CTRL>(amp, m, on, creg)))
            QSV_SLOT1(2, (reg_r1<T, R, NR, 2, CTRL>(amp, m, on, creg)))
            QSV_SLOT1(3, (reg_r1<T, R, NR, 3, CTRL>(amp, m, on, creg)))
            QSV_SLOT1(4, (reg_r1<T, R, NR, 4, CTRL>(amp, m, on, creg)))
        default: __builtin_unreachable();
        }
    } else {
        switch (j) {
            QSV_SLOT1(0, (reg_g1<T, R, NR, 0, CTRL>(amp, m, on, creg)))
            QSV_SLOT1(1, (reg_g1<T, R, NR, 1, CTRL>(amp, m, on, creg)))
            QSV_SLOT1(2, (reg_g1<T, R, NR, 2, CTRL>(amp, m, on, creg)))
            QSV_SLOT1(3, (reg_g1<T, R, NR, 3, CTRL>(amp, m, on, creg)))
            QSV_SLOT1(4, (reg_g1<T, R, NR, 4, CTRL>(amp, m, on, creg)))
        default: __builtin_unreachable();
        }
    }
}

// m16: the first 16 coefficients (all of a real 2-qubit matrix); a complex
// 2-qubit matrix reads its other 16 from the op.
template <typename T, typename R, int NR, int RB, bool CTRL>
__device__ __forceinline__ void dispatch_2(T *amp, int kind, int a, int b, const R *m16,
                                           const RegOp &op, bool on, uint32_t creg) {
#define QSV_PAIR(A, B)                                                                   \
    case (A) * 8 + (B):                                                                  \
        if constexpr (RB > (B)) {                                                        \
            if (kind == ROP_R2) {                                                        \
                reg_r2<T, R, NR, A, B, CTRL>(amp, m16, on, creg);                        \
            } else {                                                                     \
                R m32[32];                                                               \
                const R *src = op_mat<R>(op);                                            \
                _Pragma("unroll") for (int e = 0; e < 16; ++e) m32[e] = m16[e];          \
                _Pragma("unroll") for (int e = 16; e < 32; ++e) m32[e] = src[e];         \
                reg_g2<T, R, NR, A, B, CTRL>(amp, m32, on, creg);                        \
            }                                                                            \
        } else {                                                                         \
            __builtin_unreachable();                                                     \
        }                                                                                \
        break;
    switch (a * 8 + b) {
        QSV_PAIR(0, 1) QSV_PAIR(0, 2) QSV_PAIR(1, 2) QSV_PAIR(0, 3) QSV_PAIR(1, 3) QSV_PAIR(2, 3)
        QSV_PAIR(0, 4) QSV_PAIR(1, 4) QSV_PAIR(2, 4) QSV_PAIR(3, 4)
    default: __builtin_unreachable();   // the host emits only valid slot pairs
    }
#undef QSV_PAIR
}

// One operation of a register program on the thread's amplitudes.  Every
// case writes every amplitude (no skipped op or group), see reg_g1.  The
// fields every op kind may need and the first 16 matrix coefficients are
// read up front, so their scalar loads go out in one burst and the op waits
// once instead of once per dependent field.
template <typename T, typename R, int NR, int RB, bool DG>
__device__ __forceinline__ void reg_op(T *amp, const RegOp &op, uint32_t lds_a, uint32_t limg_a,
                                       uint64_t base, uint32_t lane, uint32_t wave) {
    const int kind = op.kind;
    const int a = op.a, b = op.b;
    const uint32_t creg = op.creg;
    const uint64_t octrl = op.octrl, lane_ok = op.lane_ok;
    const uint32_t wave_ok = op.wave_ok;
    const R *mp = op_mat<R>(op);
    R m16[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) m16[e] = mp[e];
    if (kind == ROP_REMAP) {
        uint32_t wr[NR], rd[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            wr[i] = op.wr[i];
            rd[i] = op.rd[i];
        }
        // the remap buffer's LDS address (a multiple of its size) joins the
        // thread parts; the register parts then XOR in
        const uint32_t lw = limg_a + op.lane_off + 4u * lane;
        const uint32_t wt = (lds_read_u32(lw) ^ op.wwave[wave]) + lds_a;
        const uint32_t rt = (lds_read_u32(lw + 256u) ^ op.rwave[wave]) + lds_a;
        // raised priority through the remap (LDS round trips and barriers
        // that the whole workgroup waits on), as for the tile's stores and
        // loads
        __builtin_amdgcn_s_setprio(2);
        switch (a) {
            QSV_SLOT1(0, (remap_half<T, NR, 0>(amp, wt, rt, wr, rd, b)))
            QSV_SLOT1(1, (remap_half<T, NR, 1>(amp, wt, rt, wr, rd, b)))
            QSV_SLOT1(2, (remap_half<T, NR, 2>(amp, wt, rt, wr, rd, b)))
            QSV_SLOT1(3, (remap_half<T, NR, 3>(amp, wt, rt, wr, rd, b)))
            QSV_SLOT1(4, (remap_half<T, NR, 4>(amp, wt, rt, wr, rd, b)))
        default: __builtin_unreachable();
        }
        __builtin_amdgcn_s_setprio(0);
    } else if (kind == ROP_DIAG) {
        if constexpr (DG) reg_diag<T, NR>(amp, op, limg_a, base, lane, wave);
        else __builtin_unreachable();
    } else if (creg == 0 && octrl == 0 && lane_ok == ~0ull && wave_ok == ~0u) {
        if (kind == ROP_G2 || kind == ROP_R2)
            dispatch_2<T, R, NR, RB, false>(amp, kind, a, b, m16, op, true, 0);
        else
            dispatch_1<T, R, NR, RB, false>(amp, kind, a, m16, true, 0);
    } else {
        // controls outside the tile (uniform), on thread-id bits (lane and
        // wave masks) and on register bits (creg)
        const bool on = ((base & octrl) == octrl) && ((wave_ok >> wave) & 1u) &&
                        ((lane_ok >> lane) & 1ull);
        if (kind == ROP_G2 || kind == ROP_R2)
            dispatch_2<T, R, NR, RB, true>(amp, kind, a, b, m16, op, on, creg);
        else
            dispatch_1<T, R, NR, RB, true>(amp, kind, a, m16, on, creg);
    }
}
#undef QSV_SLOT1

// Global index of the first amplitude of tile t: a 0 bit inserted at every
// tile position (opaque positions: their masks are not hoisted out of the
// tile loop into 2m spilled 64-bit values).
template <int M>
__device__ __forceinline__ uint64_t tile_base(uint32_t t, const TileArgs &ta) {
    uint64_t base = t;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        uint32_t tp = ta.tpos[i];
        asm volatile("" : "+s"(tp));
        const uint64_t lowm = (1ull << tp) - 1;
        base = ((base & ~lowm) << 1) | (base & lowm);
    }
    return base;
}

// Issue the loads of tile t in the load layout (this thread's part gl of the
// index).  The empty asms keep the per-register addresses and offsets from
// being hoisted out of the tile loop (as 2^RB 64-bit values they would
// spill); the offsets are a few scalar ORs per tile.
template <typename T, int RB, int M>
__device__ __forceinline__ void load_tile(T *dst, const T *__restrict__ psi, uint64_t gl,
                                          uint32_t t, const TileArgs &ta) {
    const uint64_t base = tile_base<M>(t, ta);
    const T *lp = psi + gl;
    asm volatile("" : "+v"(lp));
    lp += base;
    uint64_t gr[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) {
        gr[j] = ta.g_reg[j];
        asm volatile("" : "+s"(gr[j]));
    }
#pragma unroll
    for (int i = 0; i < (1 << RB); ++i) {
        uint64_t g = 0;
#pragma unroll
        for (int j = 0; j < RB; ++j)
            if ((i >> j) & 1) g |= gr[j];
        dst[i] = gload(lp + g);
    }
}

// Persistent: a grid of resident workgroups takes tiles from a per-pass
// counter that the host zeroes, in chunks (see below).  Dynamic LDS: the half-tile remap buffer (a workgroup remap uses all of it,
// a wave-local one its wave's share), then the pass's image (tables and
// per-lane words), copied in once per workgroup.
// DG: the instance with the diagonal-op case; programs without one run on
// the instance without it, whose register allocation the case does not
// burden.
template <typename R, int RB, int TB, bool DG>
__global__ __launch_bounds__(1 << TB) void k_tile_reg(typename VT<R>::T *__restrict__ psi,
                                                  TileArgs ta, const RegOp *__restrict__ ops,
                                                  const typename VT<R>::T *__restrict__ pool,
                                                  unsigned int *__restrict__ counter) {
    using T = typename VT<R>::T;
    constexpr int NR = 1 << RB;
    constexpr int m = RB + TB;
    constexpr uint32_t kHalf = (uint32_t)sizeof(T) << (m - 1);
    extern __shared__ __align__(16) unsigned char smem_reg[];
    unsigned char *limg = smem_reg + kHalf;
    // LDS addresses of the remap buffer and the image (the launch checks
    // that the dynamic block starts at 0, so both are multiples of kHalf)
    const uint32_t lds_a = lds_addr(smem_reg);
    const uint32_t limg_a = lds_a + kHalf;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(
            reinterpret_cast<const unsigned char *>(pool) + ta.img_off);
        uint4 *dst = reinterpret_cast<uint4 *>(limg);
        for (uint32_t e = tid; e < (ta.img_bytes >> 4); e += (1u << TB)) dst[e] = src[e];
    }
    // this thread's part of the global index in the load and the store layout
    uint64_t gl = 0, gs = 0;
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const uint64_t on = 0ull - (uint64_t)((tid >> t) & 1u);
        gl |= on & ta.g_thr[t];
        gs |= on & ta.g_thr_f[t];
    }
    const uint32_t n_tiles = (uint32_t)ta.n_tiles;

    // Tiles are claimed kChunk at a time from the pass's counter: a compute
    // unit or XCD that runs slower takes fewer chunks, and the claim is
    // broadcast through two alternating LDS slots, so one workgroup barrier
    // per chunk suffices (the slot a claim overwrites was read before the
    // barrier of the chunk in between).  Otherwise the waves of a workgroup
    // meet only at its workgroup remaps.  One tile per claim: the tiles in
    // flight across the device are then consecutive, so the 128-byte runs
    // they share a DRAM page with are fetched close together in time
    // (measured: larger chunks lose a few per cent).
    constexpr uint32_t kChunk = 1;
    // the two claim slots follow the image in dynamic LDS (a static
    // __shared__ variable would move the dynamic block off address 0, and
    // every LDS address would then take an extra add)
    uint32_t *s_claim = reinterpret_cast<uint32_t *>(limg + ta.img_bytes);
    if (tid == 0) s_claim[0] = atomicAdd(counter, kChunk);
    uint32_t slot = 0;
    uint32_t tile = 0, left = 0;
    for (;;) {
        if (left == 0) {
            __syncthreads();   // the claim (and, the first time, the image) is in LDS
            tile = __builtin_amdgcn_readfirstlane(s_claim[slot]);
            if (tile >= n_tiles) break;
            left = std::min(kChunk, n_tiles - tile);
            slot ^= 1u;
            if (tid == 0) s_claim[slot] = atomicAdd(counter, kChunk);
        }
        T amp[NR];
        load_tile<T, RB, m>(amp, psi, gl, tile, ta);
        const uint64_t base = tile_base<m>(tile, ta);
        // back to normal priority for the arithmetic (raised before the
        // stores below: a wave that stores one tile and issues the next
        // tile's loads goes ahead of the other waves' FMAs, so the memory
        // requests of the compute units go out sooner)
        __builtin_amdgcn_s_setprio(0);
        // Two ops per iteration (the host pads the program to an even
        // length): the amplitudes then alternate between two register sets
        // without copies at the loop back edge.  Op fields are read through
        // references into the uniform op array so they stay scalar.
        for (int oi = 0; oi < ta.n_ops; oi += 2) {
            reg_op<T, R, NR, RB, DG>(amp, ops[oi], lds_a, limg_a, base, lane, wave);
            reg_op<T, R, NR, RB, DG>(amp, ops[oi + 1], lds_a, limg_a, base, lane, wave);
        }
        // a pass that moves its qubits stores where other threads loaded:
        // every load of the tile completes before the first store
        if (ta.store_sync) __syncthreads();
        __builtin_amdgcn_s_setprio(2);
        T *sp = psi + gs;
        asm volatile("" : "+v"(sp));
        sp += base;
        uint64_t gr[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            gr[j] = ta.g_reg_f[j];
            asm volatile("" : "+s"(gr[j]));
        }
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            uint64_t g = 0;
#pragma unroll
            for (int j = 0; j < RB; ++j)
                if ((i >> j) & 1) g |= gr[j];
            gstore(sp + g, amp[i]);
        }
        ++tile;
        --left;
    }
}

// Batched form: one pass index of many states (segments of tiles, each
// segment one state's pass with its own program and image).  Workgroup w
// takes the contiguous items [w c, (w + 1) c), c = ceil(items / grid), so it
// mostly stays within one segment; it finds its first segment by binary
// search, steps to the next one when its items cross a segment's end, and
// reloads the image and its thread parts of the layouts at each change.
template <typename R, int RB, int TB, bool DG>
__global__ __launch_bounds__(1 << TB) void k_tile_reg_batch(typename VT<R>::T *__restrict__ states,
                                                        const RegSeg *__restrict__ segs, int nseg,
                                                        uint64_t items,
                                                        const TileArgs *__restrict__ tas,
                                                        const RegOp *__restrict__ ops,
                                                        const unsigned char *__restrict__ pool) {
    using T = typename VT<R>::T;
    constexpr int NR = 1 << RB;
    constexpr int m = RB + TB;
    constexpr uint32_t kHalf = (uint32_t)sizeof(T) << (m - 1);
    extern __shared__ __align__(16) unsigned char smem_reg[];
    unsigned char *limg = smem_reg + kHalf;
    const uint32_t lds_a = lds_addr(smem_reg);
    const uint32_t limg_a = lds_a + kHalf;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint64_t per = (items + gridDim.x - 1) / gridDim.x;
    const uint64_t it0 = (uint64_t)blockIdx.x * per;
    const uint64_t it1 = it0 + per < items ? it0 + per : items;
    int lo = 0;
    if (it0 < it1) {
        int hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segs[mid].first <= it0) lo = mid;
            else hi = mid - 1;
        }
    }
    int cur = -1;
    uint64_t gl = 0, gs = 0;
    for (uint64_t it = it0; it < it1; ++it) {
        while (lo + 1 < nseg && segs[lo + 1].first <= it) ++lo;
        const RegSeg sg = segs[lo];
        const TileArgs &ta = tas[sg.ta];
        if (lo != cur) {
            // every wave is past the previous tile (its remaps and table
            // reads) before the image is overwritten
            __syncthreads();
            const uint4 *src = reinterpret_cast<const uint4 *>(pool + ta.img_off);
            uint4 *dst = reinterpret_cast<uint4 *>(limg);
            for (uint32_t e = tid; e < (ta.img_bytes >> 4); e += (1u << TB)) dst[e] = src[e];
            gl = 0;
            gs = 0;
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const uint64_t on = 0ull - (uint64_t)((tid >> t) & 1u);
                gl |= on & ta.g_thr[t];
                gs |= on & ta.g_thr_f[t];
            }
            __syncthreads();
            cur = lo;
        }
        T *psi = states + sg.state_off;
        const uint32_t tile = (uint32_t)(it - sg.first);
        const RegOp *prog = ops + sg.op_begin;
        const int n_ops = ta.n_ops;
        T amp[NR];
        load_tile<T, RB, m>(amp, psi, gl, tile, ta);
        const uint64_t base = tile_base<m>(tile, ta);
        for (int oi = 0; oi < n_ops; oi += 2) {
            reg_op<T, R, NR, RB, DG>(amp, prog[oi], lds_a, limg_a, base, lane, wave);
            reg_op<T, R, NR, RB, DG>(amp, prog[oi + 1], lds_a, limg_a, base, lane, wave);
        }
        // stores go where other threads loaded (relabeling passes), and the
        // next tile's first workgroup remap may follow wave-local ones
        __syncthreads();
        T *sp = psi + gs;
        asm volatile("" : "+v"(sp));
        sp += base;
        uint64_t gr[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            gr[j] = ta.g_reg_f[j];
            asm volatile("" : "+s"(gr[j]));
        }
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            uint64_t g = 0;
#pragma unroll
            for (int j = 0; j < RB; ++j)
                if ((i >> j) & 1) g |= gr[j];
            gstore(sp + g, amp[i]);
        }
    }
}

template <typename R, bool DG>
static hipError_t launch_reg_batch_t(void *states, const RegSeg *segs, int nseg, uint64_t items,
                                     const TileArgs *tas, const RegOp *rops, const void *pool,
                                     uint32_t img_max, hipStream_t s) {
    using T = typename VT<R>::T;
    constexpr int RB = 4, TB = 8;
    if (items == 0 || nseg <= 0) return hipSuccess;
    if (img_max > kRegImageMax || (img_max & 15u)) return hipErrorInvalidValue;
    constexpr size_t half = sizeof(T) << (RB + TB - 1);
    const size_t lds = half + img_max;
    static bool attr = false;
    static int cus = 0;
    if (!attr) {
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_tile_reg_batch<R, RB, TB, DG>));
        if (e != hipSuccess) return e;
        if (fa.sharedSizeBytes != 0) return hipErrorInvalidDeviceFunction;
        e = set_lds_attr(k_tile_reg_batch<R, RB, TB, DG>, half + kRegImageMax);
        if (e != hipSuccess) return e;
        int dev = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        attr = true;
    }
    int occ = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, reinterpret_cast<const void *>(k_tile_reg_batch<R, RB, TB, DG>), 1 << TB, lds);
    if (e != hipSuccess) return e;
    const uint64_t resident = (uint64_t)std::max(1, cus) * (uint64_t)std::max(1, occ);
    const unsigned grid = (unsigned)std::min<uint64_t>(items, resident);
    hipLaunchKernelGGL((k_tile_reg_batch<R, RB, TB, DG>), dim3(grid), dim3(1 << TB), lds, s,
                       (T *)states, segs, nseg, items, tas, rops, (const unsigned char *)pool);
    return hipGetLastError();
}

hipError_t launch_tile_reg_batch(int dtype, bool dg, void *states, const RegSeg *segs, int nseg,
                                 uint64_t items, const TileArgs *tas, const RegOp *rops,
                                 const void *pool, uint32_t img_max, hipStream_t s) {
    if (dtype == 0)
        return dg ? launch_reg_batch_t<double, true>(states, segs, nseg, items, tas, rops, pool, img_max, s)
                  : launch_reg_batch_t<double, false>(states, segs, nseg, items, tas, rops, pool, img_max, s);
    return dg ? launch_reg_batch_t<float, true>(states, segs, nseg, items, tas, rops, pool, img_max, s)
              : launch_reg_batch_t<float, false>(states, segs, nseg, items, tas, rops, pool, img_max, s);
}

int tile_pass_max_bits(int dtype) { return dtype == 0 ? 13 : 14; }
// 16 amplitudes per thread: 64 VGPRs of state for complex128, 32 for complex64
int tile_reg_bits(int) { return 4; }

template <typename K>
static hipError_t set_lds_attr(K kern, size_t bytes) {
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

static dim3 tile_grid(uint64_t nt) {
    if (nt <= 0x7fffffffull) return dim3((unsigned)nt, 1, 1);
    return dim3(1u << 30, (unsigned)(nt >> 30), 1);
}

template <typename R, int KM>
static hipError_t launch_lds_t(void *psi, const TileArgs &ta, const TileOp *ops, const void *pool,
                               unsigned int *counter, hipStream_t s) {
    using T = typename VT<R>::T;
    const int max_bits = tile_pass_max_bits(sizeof(R) == 8 ? 0 : 1);
    static bool attr = false;
    if (!attr) {
        hipError_t e = set_lds_attr(k_tile_lds<R, KM>, (sizeof(T) << max_bits) + 16);
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (ta.n_tiles == 0) return hipSuccess;
    if (ta.n_tiles > 0xffffffffull - 65536) return hipErrorInvalidValue;
    // resident workgroups per compute unit for each tile size
    static int per_cu[16] = {0};
    static int cus = 0;
    const size_t lds = (sizeof(T) << ta.m) + 16;   // tile + counter slot
    if (per_cu[ta.m] == 0) {
        int dev = 0, occ = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess && cus == 0)
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, reinterpret_cast<const void *>(k_tile_lds<R, KM>), kNT, lds);
        if (e != hipSuccess) return e;
        per_cu[ta.m] = std::max(1, occ);
    }
    const uint64_t resident = (uint64_t)std::max(1, cus) * per_cu[ta.m];
    const unsigned grid = (unsigned)std::min<uint64_t>(ta.n_tiles, resident);
    hipLaunchKernelGGL((k_tile_lds<R, KM>), dim3(grid), dim3(kNT), lds, s, (T *)psi, ta, ops,
                       (const T *)pool, counter);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_lds_k(void *psi, const TileArgs &ta, const TileOp *ops, const void *pool,
                               unsigned int *counter, hipStream_t s) {
    switch (ta.mfma_k) {
    case 0: return launch_lds_t<R, 0>(psi, ta, ops, pool, counter, s);
    case 3: return launch_lds_t<R, 3>(psi, ta, ops, pool, counter, s);
    case 4: return launch_lds_t<R, 4>(psi, ta, ops, pool, counter, s);
    case 5: return launch_lds_t<R, 5>(psi, ta, ops, pool, counter, s);
    }
    return hipErrorInvalidValue;
}

template <typename R, int RB, int TB, bool DG>
static hipError_t launch_reg_t(void *psi, const TileArgs &ta, const RegOp *rops,
                               const void *pool, unsigned int *counter, hipStream_t s) {
    using T = typename VT<R>::T;
    if (ta.n_tiles == 0) return hipSuccess;
    if (ta.n_ops & 1) return hipErrorInvalidValue;   // programs are padded to even length
    if (ta.n_tiles > 0xffffffffull - 65536) return hipErrorInvalidValue;
    if (ta.img_bytes > kRegImageMax || (ta.img_bytes & 15u) || (ta.img_off & 15)) return hipErrorInvalidValue;
    constexpr size_t half = sizeof(T) << (RB + TB - 1);
    const size_t lds = half + ta.img_bytes + 16;   // + the two claim slots
    static int cus = 0;
    static bool attr = false;
    if (!attr) {
        // the kernel forms LDS addresses by XOR on top of the dynamic block's
        // base, which is then 0 only without static LDS
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_tile_reg<R, RB, TB, DG>));
        if (e != hipSuccess) return e;
        if (fa.sharedSizeBytes != 0) return hipErrorInvalidDeviceFunction;
        e = set_lds_attr(k_tile_reg<R, RB, TB, DG>, half + kRegImageMax + 16);
        if (e != hipSuccess) return e;
        int dev = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        attr = true;
    }
    // resident workgroups per compute unit for this image size (in 1 KiB steps)
    static int per_cu[kRegImageMax / 1024 + 2] = {0};
    const size_t slot = (ta.img_bytes + 1023) / 1024;
    if (per_cu[slot] == 0) {
        int occ = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, reinterpret_cast<const void *>(k_tile_reg<R, RB, TB, DG>), 1 << TB,
            half + slot * 1024 + 16);
        if (e != hipSuccess) return e;
        per_cu[slot] = std::max(1, occ);
    }
    const uint64_t resident = (uint64_t)std::max(1, cus) * (uint64_t)per_cu[slot];
    const unsigned grid = (unsigned)std::min<uint64_t>(ta.n_tiles, resident);
    hipLaunchKernelGGL((k_tile_reg<R, RB, TB, DG>), dim3(grid), dim3(1 << TB), lds, s, (T *)psi, ta,
                       rops, (const T *)pool, counter);
    return hipGetLastError();
}

hipError_t launch_tile_pass(int dtype, void *psi, const TileArgs &ta, const TileOp *ops,
                            const void *pool, unsigned int *counter, hipStream_t s) {
    if (ta.m < 1 || ta.m > tile_pass_max_bits(dtype)) return hipErrorInvalidValue;
    return dtype == 0 ? launch_lds_k<double>(psi, ta, ops, pool, counter, s)
                      : launch_lds_k<float>(psi, ta, ops, pool, counter, s);
}

hipError_t launch_tile_reg(int dtype, void *psi, const TileArgs &ta, const RegOp *rops,
                           const void *pool, unsigned int *counter, hipStream_t s) {
    const int rb = ta.rb, tb = ta.m - ta.rb;
#define QSV_REG_T(R, RB, TB)                                                         \
    return ta.no_diag ? launch_reg_t<R, RB, TB, false>(psi, ta, rops, pool, counter, s)   \
                      : launch_reg_t<R, RB, TB, true>(psi, ta, rops, pool, counter, s);
#define QSV_REG(R)                                                                   \
    if (tb == 8) {                                                                   \
        if (rb == 3) { QSV_REG_T(R, 3, 8) }                                          \
        if (rb == 4) { QSV_REG_T(R, 4, 8) }                                          \
        if (rb == 5) { QSV_REG_T(R, 5, 8) }                                          \
    } else if (tb == 9) {                                                            \
        if (rb == 3) { QSV_REG_T(R, 3, 9) }                                          \
        if (rb == 4) { QSV_REG_T(R, 4, 9) }                                          \
    }
    if (dtype == 0) {
        QSV_REG(double)
    } else {
        QSV_REG(float)
    }
#undef QSV_REG
#undef QSV_REG_T
    return hipErrorInvalidValue;
}

}  // namespace dev
}  // namespace qsv
