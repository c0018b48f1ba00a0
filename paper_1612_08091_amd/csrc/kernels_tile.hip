// LDS-tile passes for gfx950.  One workgroup owns a tile: the 2^m amplitudes
// whose indices agree outside the m tile bits.  The tile is read from HBM
// once, every operation of the pass is applied to it on chip, and it is
// written back once, so a pass costs one read and one write of the state
// whatever the number of gates it holds (the lazily cached gates of Sec.
// 4.3.2 executed in bulk).
//
// Two kernels:
//  * k_tile_reg<R, RB>: m = RB + 8.  Each of the 256 threads keeps 2^RB
//    amplitudes in registers.  Register bit j and thread bit i each stand for
//    one tile bit (the layout).  1- and 2-qubit dense operations on register
//    bits run in registers; diagonal operations on any bits use the global
//    index of each amplitude; a REMAP op moves the tile through LDS (XOR
//    swizzled against bank conflicts) into a new layout.  Passes holding
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
                    v[u] = psi[base | dep_tid | ta.dep_hi[(j0 >> 8) + u]];
#pragma unroll
                for (int u = 0; u < 8; ++u) tile[swz_tid ^ swz<R>(j0 + u * kNT)] = v[u];
            }
        } else {
            for (uint32_t j = 0; j < tsize; j += kNT)
                if (j + tid < tsize)
                    tile[swz_tid ^ swz<R>(j)] = psi[base | dep_tid | ta.dep_hi[j >> 8]];
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
                    psi[base | dep_tid | ta.dep_hi[(j0 >> 8) + u]] = v[u];
            }
        } else {
            for (uint32_t j = 0; j < tsize; j += kNT)
                if (j + tid < tsize)
                    psi[base | dep_tid | ta.dep_hi[j >> 8]] = tile[swz_tid ^ swz<R>(j)];
        }
        if (tid == 0) s_tile = next;
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_tile);
    }
}

// ------------------------------------------------------- k_tile_reg
template <typename T, int NR, int RB>
__device__ __forceinline__ uint64_t greg(int i, const uint64_t *gbit) {
    uint64_t g = 0;
#pragma unroll
    for (int j = 0; j < RB; ++j)
        if ((i >> j) & 1) g |= gbit[j];
    return g;
}

template <typename T, int NR, int RB, int J, bool CTRL>
__device__ __forceinline__ void reg_g1(T *amp, const T *__restrict__ U, uint64_t gb,
                                       const uint64_t *gbit, uint64_t ctrl) {
    const T u00 = U[0], u01 = U[1], u10 = U[2], u11 = U[3];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & (1 << J)) continue;
        const int i1 = i | (1 << J);
        const T a = amp[i], b = amp[i1];
        T na = cmul(u00, a);
        na = cmadd(na, u01, b);
        T nb = cmul(u10, a);
        nb = cmadd(nb, u11, b);
        if (CTRL) {
            const bool c = ((gb | greg<T, NR, RB>(i, gbit)) & ctrl) == ctrl;
            amp[i] = csel(c, na, a);
            amp[i1] = csel(c, nb, b);
        } else {
            amp[i] = na;
            amp[i1] = nb;
        }
    }
}

template <typename T, int NR, int RB, int J1, int J2, bool CTRL>
__device__ __forceinline__ void reg_g2(T *amp, const T *__restrict__ U, uint64_t gb,
                                       const uint64_t *gbit, uint64_t ctrl) {
    T u[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) u[e] = U[e];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        if (i & ((1 << J1) | (1 << J2))) continue;
        const int idx[4] = {i, i | (1 << J1), i | (1 << J2), i | (1 << J1) | (1 << J2)};
        T x[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = amp[idx[c]];
        bool c = true;
        if (CTRL) c = ((gb | greg<T, NR, RB>(i, gbit)) & ctrl) == ctrl;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T y = cmul(u[r * 4], x[0]);
#pragma unroll
            for (int cc = 1; cc < 4; ++cc) y = cmadd(y, u[r * 4 + cc], x[cc]);
            amp[idx[r]] = CTRL ? csel(c, y, x[r]) : y;
        }
    }
}

// Diagonal op: amplitude i of the thread takes the factor val[r], where the
// row index r = r_thr ^ op.wr[i] splits into the bits of the targets that
// are not register bits (read once per thread from its global base gb;
// op.pad0 marks them) and the bits from the register index (op.wr[i],
// precomputed on the host for the current layout).  Controls that are not
// register bits are in op.ctrl; those that are, as register-index bits, in
// op.b.  The wave first copies the op's 2^k factors into its own LDS table
// `tab` (every lane takes part, before any lane leaves on its controls), so
// the 16 gathers per thread are LDS reads instead of vector-memory reads
// that compete with the tile loads.  LDS operations of one wave are
// performed in order, so the reads see the copy and the next op's copy
// comes after these reads.
template <typename T, int NR, int RB>
__device__ __forceinline__ void reg_diag(T *amp, const RegOp &op, const T *__restrict__ pool,
                                         uint64_t gb, T *tab) {
    const int k = op.a;
    const uint32_t lane = threadIdx.x & 63u;
    const T *val = pool + op.mat;
    for (uint32_t e = lane; e < (1u << k); e += 64) tab[e] = val[e];
    __builtin_amdgcn_wave_barrier();
    if ((gb & op.ctrl) != op.ctrl) return;
    const uint32_t thr_targets = op.pad0;
    uint32_t rt = 0;
    for (int q = 0; q < k; ++q)
        if ((thr_targets >> q) & 1u) rt |= (uint32_t)((gb >> op.gt[q]) & 1u) << q;
    const int creg = op.b;
    // rows outside the register controls take the factor 1
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const T v = tab[rt ^ op.wr[i]];
        const bool on = (i & creg) == creg;
        T f;
        f.x = on ? v.x : decltype(v.x)(1);
        f.y = on ? v.y : decltype(v.y)(0);
        amp[i] = cmul(f, amp[i]);
    }
}

// Layout change through an LDS buffer of half a tile.  Slot J holds the same
// tile bit before and after, and the buffer drops that bit from the index.
// In phase p every thread writes its registers whose slot-J bit is p, then
// reads the same register indices in the new layout, so no register is
// overwritten before it was written out.  Addresses are the thread part XOR
// the (uniform) register part, both precomputed on the host.
template <typename T, int NR, int J>
__device__ __forceinline__ void remap_half(T *amp, unsigned char *lds, uint32_t wt, uint32_t rt,
                                           const RegOp &op) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (((i >> J) & 1) != p) continue;
            *reinterpret_cast<T *>(lds + (wt ^ op.wr[i])) = amp[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (((i >> J) & 1) != p) continue;
            amp[i] = *reinterpret_cast<const T *>(lds + (rt ^ op.rd[i]));
        }
        __syncthreads();
    }
}

template <typename T, int NR, int RB, bool CTRL>
__device__ __forceinline__ void dispatch_g1(T *amp, int j, const T *U, uint64_t gb,
                                            const uint64_t *gbit, uint64_t ctrl) {
    switch (j) {
    case 0: reg_g1<T, NR, RB, 0, CTRL>(amp, U, gb, gbit, ctrl); break;
    case 1: reg_g1<T, NR, RB, 1, CTRL>(amp, U, gb, gbit, ctrl); break;
    case 2: reg_g1<T, NR, RB, 2, CTRL>(amp, U, gb, gbit, ctrl); break;
    case 3:
        if constexpr (RB > 3) reg_g1<T, NR, RB, 3, CTRL>(amp, U, gb, gbit, ctrl);
        else __builtin_unreachable();
        break;
    case 4:
        if constexpr (RB > 4) reg_g1<T, NR, RB, 4, CTRL>(amp, U, gb, gbit, ctrl);
        else __builtin_unreachable();
        break;
    default: __builtin_unreachable();   // the host emits only valid slots
    }
}

template <typename T, int NR, int RB, bool CTRL>
__device__ __forceinline__ void dispatch_g2(T *amp, int a, int b, const T *U, uint64_t gb,
                                            const uint64_t *gbit, uint64_t ctrl) {
#define QSV_G2(A, B) \
    case (A) * 8 + (B): reg_g2<T, NR, RB, A, B, CTRL>(amp, U, gb, gbit, ctrl); break;
    switch (a * 8 + b) {
        QSV_G2(0, 1) QSV_G2(0, 2) QSV_G2(1, 2)
    default:
        if constexpr (RB == 4) {
            switch (a * 8 + b) {
                QSV_G2(0, 3) QSV_G2(1, 3) QSV_G2(2, 3)
            default: __builtin_unreachable();
            }
        } else if constexpr (RB == 5) {
            switch (a * 8 + b) {
                QSV_G2(0, 3) QSV_G2(1, 3) QSV_G2(2, 3) QSV_G2(0, 4) QSV_G2(1, 4) QSV_G2(2, 4)
                QSV_G2(3, 4)
            default: __builtin_unreachable();
            }
        } else {
            __builtin_unreachable();
        }
        break;
    }
#undef QSV_G2
}

// One operation of a register program on the thread's amplitudes.
template <typename T, int NR, int RB, int TB, bool DG>
__device__ __forceinline__ void reg_op(T *amp, const RegOp &op, const T *__restrict__ pool,
                                       unsigned char *lds, T *dtab, uint64_t base, uint64_t &gthr,
                                       uint64_t *gbit, uint32_t tid) {
    const int kind = op.kind;
    const uint64_t gb = base | gthr;
    if (kind == ROP_G1) {
        const T *U = pool + op.mat;
        if (op.ctrl) dispatch_g1<T, NR, RB, true>(amp, op.a, U, gb, gbit, op.ctrl);
        else dispatch_g1<T, NR, RB, false>(amp, op.a, U, gb, gbit, 0);
    } else if (kind == ROP_G2) {
        const T *U = pool + op.mat;
        if (op.ctrl) dispatch_g2<T, NR, RB, true>(amp, op.a, op.b, U, gb, gbit, op.ctrl);
        else dispatch_g2<T, NR, RB, false>(amp, op.a, op.b, U, gb, gbit, 0);
    } else if (kind == ROP_DIAG) {
        if constexpr (DG) reg_diag<T, NR, RB>(amp, op, pool, gb, dtab);
        else __builtin_unreachable();
    } else {
        // thread parts from the thread-id bits; the empty asm makes the id
        // opaque so the per-bit masks are not kept live across the op loop
        uint32_t tr = tid;
        asm volatile("" : "+v"(tr));
        uint32_t wt = 0, rt = 0;
        uint64_t gthr_n = 0;
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const uint32_t msk = 0u - ((tr >> t) & 1u);
            wt ^= msk & op.wthr[t];
            rt ^= msk & op.rthr[t];
            gthr_n |= (((uint64_t)msk << 32) | msk) & op.g_thr[t];
        }
        // raised priority through the remap (LDS round trips and barriers
        // that the whole workgroup waits on), as for the tile's stores and
        // loads
        __builtin_amdgcn_s_setprio(2);
        switch (op.a) {
        case 0: remap_half<T, NR, 0>(amp, lds, wt, rt, op); break;
        case 1: remap_half<T, NR, 1>(amp, lds, wt, rt, op); break;
        case 2: remap_half<T, NR, 2>(amp, lds, wt, rt, op); break;
        case 3:
            if constexpr (RB > 3) remap_half<T, NR, 3>(amp, lds, wt, rt, op);
            else __builtin_unreachable();
            break;
        case 4:
            if constexpr (RB > 4) remap_half<T, NR, 4>(amp, lds, wt, rt, op);
            else __builtin_unreachable();
            break;
        default: __builtin_unreachable();
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int j = 0; j < RB; ++j) gbit[j] = op.g_reg[j];
        gthr = gthr_n;
    }
}

// Persistent: a grid of resident workgroups takes tiles from an atomic
// counter (one per pass, zeroed by the host upload), so a compute unit or XCD
// that runs slower simply processes fewer tiles and no dispatch gaps open up
// between tiles.  Every workgroup leaves once the counter has passed the tile
// count.
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
    // half a tile for the two-phase remaps (static, so addresses need no base)
    __shared__ T half_tile[1 << (m - 1)];
    __shared__ unsigned int s_tile;
    // one table of diagonal factors (at most 2^kRegDiagMax) per wave
    constexpr int kTab = 1 << kRegDiagMax;
    __shared__ T diag_tab[DG ? ((1 << TB) >> 6) * kTab : 1];
    unsigned char *lds = reinterpret_cast<unsigned char *>(half_tile);
    const uint32_t tid = threadIdx.x;
    T *dtab = diag_tab + (DG ? (tid >> 6) * kTab : 0);
    // layout at load time (the same for every tile): global index bit of each
    // register bit (uniform) and the global bits of this thread
    uint64_t gbit0[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) gbit0[j] = ta.g_reg[j];
    uint64_t gthr0 = 0;
#pragma unroll
    for (int t = 0; t < TB; ++t) gthr0 |= (0ull - ((tid >> t) & 1u)) & ta.g_thr[t];
    const uint32_t n_tiles = (uint32_t)ta.n_tiles;

    if (tid == 0) s_tile = atomicAdd(counter, 1u);
    __syncthreads();
    uint32_t tile = __builtin_amdgcn_readfirstlane(s_tile);
    while (tile < n_tiles) {
        uint64_t base = tile;
#pragma unroll
        for (int i = 0; i < m; ++i) {
            const uint64_t lowm = (1ull << ta.tpos[i]) - 1;
            base = ((base & ~lowm) << 1) | (base & lowm);
        }
        // the empty asm keeps the per-register load addresses from being
        // hoisted out of the tile loop (32 VGPRs held for its whole life)
        uint64_t gthr = gthr0;
        asm volatile("" : "+v"(gthr));
        T amp[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) amp[i] = psi[base | gthr | greg<T, NR, RB>(i, gbit0)];
        // claim the next tile now; the atomic's latency hides behind the ops
        unsigned int next = 0;
        if (tid == 0) next = atomicAdd(counter, 1u);
        // back to normal priority for the arithmetic (raised before the
        // stores below: a wave that stores one tile and issues the next
        // tile's loads goes ahead of the other waves' FMAs, so the memory
        // requests of the compute units go out sooner)
        __builtin_amdgcn_s_setprio(0);
        uint64_t gbit[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) gbit[j] = gbit0[j];
        // Two ops per iteration (the host pads the program to an even length
        // with an identity 1-qubit op): the amplitudes then alternate between
        // two register sets without copies at the loop back edge.  Op fields
        // are read through references into the uniform op array so they stay
        // scalar.
        for (int oi = 0; oi < ta.n_ops; oi += 2) {
            reg_op<T, NR, RB, TB, DG>(amp, ops[oi], pool, lds, dtab, base, gthr, gbit, tid);
            reg_op<T, NR, RB, TB, DG>(amp, ops[oi + 1], pool, lds, dtab, base, gthr, gbit, tid);
        }
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int i = 0; i < NR; ++i) psi[base | gthr | greg<T, NR, RB>(i, gbit)] = amp[i];
        __syncthreads();   // every thread has read s_tile and left the LDS buffer
        if (tid == 0) s_tile = next;
        __syncthreads();
        tile = __builtin_amdgcn_readfirstlane(s_tile);
    }
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
    static unsigned resident = 0;   // workgroups the device holds at once
    if (resident == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void *>(k_tile_reg<R, RB, TB, DG>), 1 << TB, 0);
        if (e != hipSuccess) return e;
        resident = (unsigned)std::max(1, cus * std::max(1, per_cu));
    }
    const unsigned grid = (unsigned)std::min<uint64_t>(ta.n_tiles, resident);
    hipLaunchKernelGGL((k_tile_reg<R, RB, TB, DG>), dim3(grid), dim3(1 << TB), 0, s, (T *)psi, ta,
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
