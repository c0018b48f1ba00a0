// Tiled reverse sweep of the adjoint gradient: psi and phi tiles in LDS, the
// reverse steps of one pass applied to both, and the rotation gradients
// Im<phi|P|psi> accumulated per workgroup and wave.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "adjoint_tile.hpp"
#include "lds_ops.hpp"

namespace qsv {
namespace dev {

// v from the lane that DPP control `ctrl` selects (per 32-bit half).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes (the same value in every lane): within each row of
// 16 lanes by DPP (swap neighbours, swap pairs, rotate by 4, rotate by 8),
// then the four row sums read from lanes 0, 16, 32 and 48.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<0xb1>(v);    // quad_perm(1, 0, 3, 2)
    v += dpp_d<0x4e>(v);    // quad_perm(2, 3, 0, 1)
    v += dpp_d<0x124>(v);   // row_ror:4
    v += dpp_d<0x128>(v);   // row_ror:8
    return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

// ------------------------------------------------ steps on the two tiles
// As the forward LDS ops (group g = threadIdx.x + kNT * it, addresses from
// the op's byte offsets), but on both tiles at once and with the loads of G
// groups issued before any of their stores, so that a wave has the reads of
// G groups of both tiles in flight instead of one group's.

// Dense (MONO = false: D x D matrix) or monomial (MONO = true: row r takes
// val[r] times row perm[r]; untouched rows are left alone) op of K targets.
template <typename R, int K, bool MONO, int G>
__device__ __forceinline__ void step_groups(unsigned char *tp, unsigned char *tf,
                                            const uint32_t *go, const uint32_t *sl,
                                            const uint32_t *ss, uint32_t touch,
                                            const typename VT<R>::T *u) {
    using T = typename VT<R>::T;
    constexpr int D = 1 << K;
    T x[G][D], y[G][D];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int r = 0; r < D; ++r) {
            if (MONO && !((touch >> r) & 1)) continue;
            const uint32_t a = go[g] ^ (MONO ? ss[r] : sl[r]);
            x[g][r] = *reinterpret_cast<const T *>(tp + a);
            y[g][r] = *reinterpret_cast<const T *>(tf + a);
        }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int r = 0; r < D; ++r) {
            if (MONO && !((touch >> r) & 1)) continue;
            T xo, yo;
            if (MONO) {
                xo = cmul(u[r], x[g][r]);
                yo = cmul(u[r], y[g][r]);
            } else {
                xo = cmul(u[r * D], x[g][0]);
                yo = cmul(u[r * D], y[g][0]);
#pragma unroll
                for (int c = 1; c < D; ++c) {
                    xo = cmadd(xo, u[r * D + c], x[g][c]);
                    yo = cmadd(yo, u[r * D + c], y[g][c]);
                }
            }
            const uint32_t a = go[g] ^ sl[r];
            *reinterpret_cast<T *>(tp + a) = xo;
            *reinterpret_cast<T *>(tf + a) = yo;
        }
}

template <typename R, int K, bool MONO, int G>
__device__ __forceinline__ void lds2_step(unsigned char *tp, unsigned char *tf, const TileOp &op,
                                          const typename VT<R>::T *__restrict__ mat) {
    using T = typename VT<R>::T;
    constexpr int D = 1 << K;
    const int nfree = op.nfree;
    const uint32_t ngroups = 1u << nfree;
    const uint32_t tid = threadIdx.x;
    const uint32_t toff = xor_parts(tid, op.fz, nfree < 8 ? nfree : 8);
    const Parts<8> hi(op.fz + 8, nfree - 8);
    const uint32_t touch = MONO ? op.touch : 0u;
    uint32_t sl[D], ss[D];
    T u[MONO ? D : D * D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        sl[r] = op.sl[r];
        ss[r] = MONO ? op.ss[r] : 0u;
    }
#pragma unroll
    for (int e = 0; e < (MONO ? D : D * D); ++e) u[e] = mat[e];
    if (ngroups >= (uint32_t)(G * kNT)) {
        // it is a multiple of G, so hi.of(it + g) = hi.of(it) ^ hi.of(g)
        uint32_t hg[G];
#pragma unroll
        for (int g = 0; g < G; ++g) hg[g] = toff ^ hi.of(g);
        for (uint32_t it = 0; it * kNT < ngroups; it += G) {
            const uint32_t hit = hi.of(it);
            uint32_t go[G];
#pragma unroll
            for (int g = 0; g < G; ++g) go[g] = hg[g] ^ hit;
            step_groups<R, K, MONO, G>(tp, tf, go, sl, ss, touch, u);
        }
    } else {
        for (uint32_t it = 0; it * kNT < ngroups; ++it) {
            if (tid >= ngroups) break;
            const uint32_t go = toff ^ hi.of(it);
            step_groups<R, K, MONO, 1>(tp, tf, &go, sl, ss, touch, u);
        }
    }
}

// U^dagger = c + i s P of one rotation on the pair (a0, a1).
template <typename T, typename R>
__device__ __forceinline__ void rot_apply(int axis, R c, R s, T &a0, T &a1) {
    T b0, b1;
    if (axis == 1) {          // i s X
        b0.x = c * a0.x - s * a1.y;
        b0.y = c * a0.y + s * a1.x;
        b1.x = c * a1.x - s * a0.y;
        b1.y = c * a1.y + s * a0.x;
    } else if (axis == 2) {   // i s Y = [[0, s], [-s, 0]]
        b0.x = c * a0.x + s * a1.x;
        b0.y = c * a0.y + s * a1.y;
        b1.x = c * a1.x - s * a0.x;
        b1.y = c * a1.y - s * a0.y;
    } else {                  // i s Z = diag(i s, -i s)
        b0.x = c * a0.x - s * a0.y;
        b0.y = c * a0.y + s * a0.x;
        b1.x = c * a1.x + s * a1.y;
        b1.y = c * a1.y - s * a1.x;
    }
    a0 = b0;
    a1 = b1;
}

// Im(conj(y0) (P x)_0 + conj(y1) (P x)_1) in double.
template <typename T>
__device__ __forceinline__ double rot_grad(int axis, const T &x0, const T &x1, const T &y0,
                                           const T &y1) {
    auto im = [](const T &a, const T &b) {   // Im(conj(a) b)
        return (double)a.x * (double)b.y - (double)a.y * (double)b.x;
    };
    auto re = [](const T &a, const T &b) {   // Re(conj(a) b)
        return (double)a.x * (double)b.x + (double)a.y * (double)b.y;
    };
    if (axis == 1) return im(y0, x1) + im(y1, x0);       // P x = (x1, x0)
    if (axis == 2) return re(y1, x0) - re(y0, x1);       // P x = (-i x1, i x0)
    return im(y0, x0) - im(y1, x1);                      // P x = (x0, -x1)
}

template <typename R, int G>
__device__ __forceinline__ void chain_groups(unsigned char *tp, unsigned char *tf,
                                             const uint32_t *go, uint32_t s0, uint32_t s1,
                                             int nsub, const int *axis, const R *c, const R *s,
                                             double *part) {
    using T = typename VT<R>::T;
    T x0[G], x1[G], y0[G], y1[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        x0[g] = *reinterpret_cast<const T *>(tp + (go[g] ^ s0));
        x1[g] = *reinterpret_cast<const T *>(tp + (go[g] ^ s1));
        y0[g] = *reinterpret_cast<const T *>(tf + (go[g] ^ s0));
        y1[g] = *reinterpret_cast<const T *>(tf + (go[g] ^ s1));
    }
#pragma unroll
    for (int j = 0; j < kAdjChain; ++j) {
        if (j >= nsub) break;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            part[j] += rot_grad(axis[j], x0[g], x1[g], y0[g], y1[g]);
            rot_apply(axis[j], c[j], s[j], x0[g], x1[g]);
            rot_apply(axis[j], c[j], s[j], y0[g], y1[g]);
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        *reinterpret_cast<T *>(tp + (go[g] ^ s0)) = x0[g];
        *reinterpret_cast<T *>(tp + (go[g] ^ s1)) = x1[g];
        *reinterpret_cast<T *>(tf + (go[g] ^ s0)) = y0[g];
        *reinterpret_cast<T *>(tf + (go[g] ^ s1)) = y1[g];
    }
}

// A rotation chain (kind ADJ_ROT); part[j] gets this thread's share of the
// j-th inner product.
template <typename R>
__device__ __forceinline__ void lds2_chain(unsigned char *tp, unsigned char *tf, const AdjOp &ao,
                                           double *part) {
    constexpr int G = 4;
    const TileOp &op = ao.op;
    const int nfree = op.nfree;
    const uint32_t ngroups = 1u << nfree;
    const uint32_t tid = threadIdx.x;
    const uint32_t toff = xor_parts(tid, op.fz, nfree < 8 ? nfree : 8);
    const Parts<8> hi(op.fz + 8, nfree - 8);
    const uint32_t s0 = op.sl[0], s1 = op.sl[1];
    const int nsub = ao.nsub;
    int axis[kAdjChain];
    R c[kAdjChain], s[kAdjChain];
#pragma unroll
    for (int j = 0; j < kAdjChain; ++j) {
        axis[j] = ao.axis[j];
        c[j] = (R)ao.c[j];
        s[j] = (R)ao.s[j];
    }
    if (ngroups >= (uint32_t)(G * kNT)) {
        uint32_t hg[G];
#pragma unroll
        for (int g = 0; g < G; ++g) hg[g] = toff ^ hi.of(g);
        for (uint32_t it = 0; it * kNT < ngroups; it += G) {
            const uint32_t hit = hi.of(it);
            uint32_t go[G];
#pragma unroll
            for (int g = 0; g < G; ++g) go[g] = hg[g] ^ hit;
            chain_groups<R, G>(tp, tf, go, s0, s1, nsub, axis, c, s, part);
        }
    } else {
        for (uint32_t it = 0; it * kNT < ngroups; ++it) {
            if (tid >= ngroups) break;
            const uint32_t go = toff ^ hi.of(it);
            chain_groups<R, 1>(tp, tf, &go, s0, s1, nsub, axis, c, s, part);
        }
    }
}

// A diagonal step whose targets all lie outside the tile (kind ADJ_PHASE):
// on this tile it multiplies the amplitudes whose in-tile control bits are
// set by one phase, val[r], r from the target bits of the tile's base index.
// Without in-tile controls that phase is the same for the whole tile and for
// both vectors, so it is only recorded in `pend` and applied when the tiles
// are written back (a common phase of both tiles changes no inner product
// Im<phi|P|psi> taken on them in between).
template <typename R>
__device__ __forceinline__ void lds2_phase(unsigned char *tp, unsigned char *tf, int m,
                                           uint64_t base, const TileOp &op,
                                           const typename VT<R>::T *__restrict__ val,
                                           typename VT<R>::T &pend) {
    using T = typename VT<R>::T;
    uint32_t r = 0;
    for (int q = 0; q < op.k; ++q) r |= (uint32_t)((base >> op.gt[q]) & 1u) << q;
    if (!((op.touch >> r) & 1u)) return;
    const T p = val[r];
    const int nfree = op.nfree;
    if (nfree == m) {
        pend = cmul(pend, p);
        return;
    }
    const uint32_t ngroups = 1u << nfree;
    const uint32_t tid = threadIdx.x;
    const uint32_t toff = xor_parts(tid, op.fz, nfree < 8 ? nfree : 8);
    const Parts<8> hi(op.fz + 8, nfree - 8);
    const uint32_t s0 = op.sl[0];
    for (uint32_t it = 0; it * kNT < ngroups; ++it) {
        if (tid >= ngroups) break;
        const uint32_t a = toff ^ hi.of(it) ^ s0;
        T *x = reinterpret_cast<T *>(tp + a);
        T *y = reinterpret_cast<T *>(tf + a);
        const T xv = *x, yv = *y;
        *x = cmul(p, xv);
        *y = cmul(p, yv);
    }
}

// ------------------------------------------------------------ blocks
// Sub-steps on the 8 rows of one group held in registers (x: psi, y: phi).
// J (block bit) and AX (rotation axis) are template arguments so that every
// row index is a compile-time constant and the rows stay in registers.
// Rows of the p-th pair (p = 0..3) on block bit J: bit J of the row
// inserted as 0 (lo) or 1 (hi).
template <int J> __device__ constexpr int pair_lo(int p) {
    return (p & ((1 << J) - 1)) | ((p >> J) << (J + 1));
}

template <typename T, typename R, int J, int AX, bool CTRL>
__device__ __forceinline__ double blk_rot(T *x, T *y, int cmask, R c, R s) {
    double part = 0.0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int r0 = pair_lo<J>(p), r1 = r0 | (1 << J);
        if (CTRL && (r0 & cmask) != cmask) continue;
        part += rot_grad(AX, x[r0], x[r1], y[r0], y[r1]);
        rot_apply(AX, c, s, x[r0], x[r1]);
        rot_apply(AX, c, s, y[r0], y[r1]);
    }
    return part;
}

template <typename T, int J>
__device__ __forceinline__ void blk_u1(T *x, T *y, int cmask, const T *u) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int r0 = pair_lo<J>(p), r1 = r0 | (1 << J);
        if ((r0 & cmask) != cmask) continue;
        const T x0 = x[r0], x1 = x[r1], y0 = y[r0], y1 = y[r1];
        x[r0] = cmadd(cmul(u[0], x0), u[1], x1);
        x[r1] = cmadd(cmul(u[2], x0), u[3], x1);
        y[r0] = cmadd(cmul(u[0], y0), u[1], y1);
        y[r1] = cmadd(cmul(u[2], y0), u[3], y1);
    }
}

template <typename T>
__device__ __forceinline__ void blk_scale(T *x, T *y, uint32_t rows, const T *d, bool same) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        if (!((rows >> r) & 1u)) continue;
        const T f = same ? d[0] : d[r];
        x[r] = cmul(f, x[r]);
        y[r] = cmul(f, y[r]);
    }
}

template <typename T, typename R, int J>
__device__ __forceinline__ double blk_rot_axis(T *x, T *y, int axis, int cmask, R c, R s) {
    // (without in-block controls every pair takes part: no per-pair tests)
    if (cmask == 0) {
        if (axis == 1) return blk_rot<T, R, J, 1, false>(x, y, 0, c, s);
        if (axis == 2) return blk_rot<T, R, J, 2, false>(x, y, 0, c, s);
        return blk_rot<T, R, J, 3, false>(x, y, 0, c, s);
    }
    if (axis == 1) return blk_rot<T, R, J, 1, true>(x, y, cmask, c, s);
    if (axis == 2) return blk_rot<T, R, J, 2, true>(x, y, cmask, c, s);
    return blk_rot<T, R, J, 3, true>(x, y, cmask, c, s);
}

// A block step.  Each thread takes groups tid, tid + kNT, ... one at a time
// (all sub-steps on one group, then the next).  With fewer than kNT groups
// the idle lanes hold zeros, which add nothing to the inner products, and
// store nothing; every lane takes part in the wave sums.
template <typename R>
__device__ __forceinline__ void lds2_block(unsigned char *tp, unsigned char *tf, uint64_t base,
                                           const AdjOp &ao, const AdjSub *__restrict__ subs,
                                           const typename VT<R>::T *__restrict__ pool,
                                           double *acc, typename VT<R>::T &pend) {
    using T = typename VT<R>::T;
    const TileOp &op = ao.op;
    const int nfree = op.nfree;
    const uint32_t ngroups = 1u << nfree;
    const uint32_t tid = threadIdx.x;
    const bool valid = tid < ngroups;
    const uint32_t toff = xor_parts(tid, op.fz, nfree < 8 ? nfree : 8);
    const Parts<8> hi(op.fz + 8, nfree - 8);
    uint32_t sl[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) sl[r] = op.sl[r];
    const uint32_t wave = tid >> 6;
    const int nsub = ao.nsub;
    const AdjSub *sb = subs + ao.sub0;
    // the pending phase is uniform: record it on the first group only
    bool first = true;
    for (uint32_t it = 0; it * kNT < ngroups || it == 0; ++it) {
        const uint32_t go = toff ^ hi.of(it);
        T x[8], y[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (valid) {
                x[r] = *reinterpret_cast<const T *>(tp + (go ^ sl[r]));
                y[r] = *reinterpret_cast<const T *>(tf + (go ^ sl[r]));
            } else {
                x[r].x = x[r].y = y[r].x = y[r].y = R(0);
            }
        }
        for (int si = 0; si < nsub; ++si) {
            const AdjSub &u = sb[si];
            if ((base & u.ectrl) != u.ectrl) continue;
            const int kind = u.kind;
            if (kind == SUB_ROT) {
                const int j = u.j, axis = u.axis, cmask = u.cmask;
                const R c = (R)u.c, s = (R)u.s;
                double part;
                if (j == 0) part = blk_rot_axis<T, R, 0>(x, y, axis, cmask, c, s);
                else if (j == 1) part = blk_rot_axis<T, R, 1>(x, y, axis, cmask, c, s);
                else part = blk_rot_axis<T, R, 2>(x, y, axis, cmask, c, s);
                const double tot = wave_sum(part);
                // (the slot belongs to this wave; an atomic add needs no
                // read-back wait before the next sub-step)
                if ((tid & 63u) == 0) atomicAdd(&acc[u.lslot * kAdjWaves + wave], tot);
            } else if (kind == SUB_U1) {
                const int j = u.j, cmask = u.cmask;
                const T *m = pool + u.mat;
                T um[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) um[e] = m[e];
                if (j == 0) blk_u1<T, 0>(x, y, cmask, um);
                else if (j == 1) blk_u1<T, 1>(x, y, cmask, um);
                else blk_u1<T, 2>(x, y, cmask, um);
            } else if (kind == SUB_DIAG) {
                const uint32_t touch = u.touch;
                const T *m = pool + u.mat;
                T d[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) d[r] = ((touch >> r) & 1u) ? m[r] : T{};
                blk_scale(x, y, touch, d, false);
            } else {
                uint32_t r = 0;
                for (int q = 0; q < u.k; ++q) r |= (uint32_t)((base >> u.gt[q]) & 1u) << q;
                if (!((u.touch >> r) & 1u)) continue;
                const T p = pool[u.mat + r];
                const int cmask = u.cmask;
                if (cmask == 0) {
                    if (first) pend = cmul(pend, p);
                    continue;
                }
                uint32_t rows = 0;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if ((q & cmask) == cmask) rows |= 1u << q;
                blk_scale(x, y, rows, &p, true);
            }
        }
        if (valid) {
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                *reinterpret_cast<T *>(tp + (go ^ sl[r])) = x[r];
                *reinterpret_cast<T *>(tf + (go ^ sl[r])) = y[r];
            }
        }
        first = false;
    }
}

// One step; returns false if it did not touch the tiles in LDS (a pending
// tile phase), so that no barrier is needed after it.
template <typename R, int KM>
__device__ __forceinline__ bool adj_step(typename VT<R>::T *tp, typename VT<R>::T *tf, int m,
                                         uint64_t base, const TileArgs &ta, const AdjOp &ao,
                                         const AdjSub *__restrict__ subs,
                                         const typename VT<R>::T *__restrict__ pool,
                                         double *acc, typename VT<R>::T &pend) {
    unsigned char *bp = reinterpret_cast<unsigned char *>(tp);
    unsigned char *bf = reinterpret_cast<unsigned char *>(tf);
    const TileOp &op = ao.op;
    if (ao.kind == ADJ_BLOCK) {
        lds2_block<R>(bp, bf, base, ao, subs, pool, acc, pend);
        return true;
    }
    if (ao.kind == ADJ_PHASE && op.nfree == m) {
        if ((base & op.ectrl) == op.ectrl)
            lds2_phase<R>(bp, bf, m, base, op, pool + op.mat, pend);
        return false;
    }
    if ((base & op.ectrl) != op.ectrl) return true;
    if (ao.kind == ADJ_ROT) {
        double part[kAdjChain] = {0.0, 0.0, 0.0, 0.0};
        lds2_chain<R>(bp, bf, ao, part);
        const uint32_t wave = threadIdx.x >> 6;
        const int nsub = ao.nsub;
        double tot[kAdjChain];
#pragma unroll
        for (int j = 0; j < kAdjChain; ++j)
            if (j < nsub) tot[j] = wave_sum(part[j]);
        if ((threadIdx.x & 63u) == 0) {
#pragma unroll
            for (int j = 0; j < kAdjChain; ++j)
                if (j < nsub) acc[ao.lslot[j] * kAdjWaves + wave] += tot[j];
        }
        return true;
    }
    const typename VT<R>::T *mat = pool + op.mat;
    if (ao.kind == ADJ_PHASE) {
        lds2_phase<R>(bp, bf, m, base, op, mat, pend);
    } else if (op.kind == TOP_DENSE && op.k == 1) {
        lds2_step<R, 1, false, 4>(bp, bf, op, mat);
    } else if (op.kind == TOP_DENSE && op.k == 2) {
        lds2_step<R, 2, false, 2>(bp, bf, op, mat);
    } else if (op.kind == TOP_MONO && op.k == 1) {
        lds2_step<R, 1, true, 4>(bp, bf, op, mat);
    } else if (op.kind == TOP_MONO && op.k == 2) {
        lds2_step<R, 2, true, 2>(bp, bf, op, mat);
    } else if (op.kind == TOP_MONO && op.k == 3) {
        lds2_step<R, 3, true, 1>(bp, bf, op, mat);
    } else {
        // matrix-core ops and diagonal ops with targets on both sides of the
        // tile boundary: the forward tile code, once per tile
        lds_op<R, KM>(tp, m, base, ta.tpos, op, pool, ta.dep_hi);
        lds_op<R, KM>(tf, m, base, ta.tpos, op, pool, ta.dep_hi);
    }
    return true;
}

// Tiles t = blockIdx.x, blockIdx.x + gridDim.x, ... (a static assignment, so
// that every partial sum is formed in the same order on every run).
// Dynamic LDS: [psi tile][phi tile][acc: kAdjMaxRot x kAdjWaves doubles].
template <typename R, int KM>
__global__ __launch_bounds__(kNT) void k_adj_tile(typename VT<R>::T *__restrict__ psi,
                                                  typename VT<R>::T *__restrict__ phi,
                                                  TileArgs ta, const AdjOp *__restrict__ ops,
                                                  const AdjSub *__restrict__ subs,
                                                  const typename VT<R>::T *__restrict__ pool,
                                                  int nrot, double *__restrict__ partial) {
    using T = typename VT<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int m = ta.m;
    const uint32_t tsize = 1u << m;
    T *tp = reinterpret_cast<T *>(smem_raw);
    T *tf = tp + tsize;
    double *acc = reinterpret_cast<double *>(tf + tsize);
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < (uint32_t)(nrot * kAdjWaves); i += kNT) acc[i] = 0.0;
    const uint64_t dep_tid = deposit_bits(tid & (tsize - 1), ta.tpos, m);
    const uint32_t swz_tid = swz<R>(tid & (tsize - 1));
    const uint64_t n_tiles = ta.n_tiles;
    for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        uint64_t base = t;
        for (int i = 0; i < m; ++i) {
            const uint64_t lowm = (1ull << ta.tpos[i]) - 1;
            base = ((base & ~lowm) << 1) | (base & lowm);
        }
        if (tsize >= 4 * kNT) {
            for (uint32_t j0 = 0; j0 < tsize; j0 += 4 * kNT) {
                T v[4], w[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint64_t gi = base | dep_tid | ta.dep_hi[(j0 >> 8) + u];
                    v[u] = psi[gi];
                    w[u] = phi[gi];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t li = swz_tid ^ swz<R>(j0 + u * kNT);
                    tp[li] = v[u];
                    tf[li] = w[u];
                }
            }
        } else {
            for (uint32_t j = 0; j < tsize; j += kNT)
                if (j + tid < tsize) {
                    const uint64_t gi = base | dep_tid | ta.dep_hi[j >> 8];
                    const uint32_t li = swz_tid ^ swz<R>(j);
                    tp[li] = psi[gi];
                    tf[li] = phi[gi];
                }
        }
        // normal priority for the steps; raised for the stores and the next
        // tiles' loads, which then go out ahead of other waves' arithmetic
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        T pend;
        pend.x = R(1);
        pend.y = R(0);
        for (int oi = 0; oi < ta.n_ops; ++oi)
            if (adj_step<R, KM>(tp, tf, m, base, ta, ops[oi], subs, pool, acc, pend))
                __syncthreads();
        __builtin_amdgcn_s_setprio(2);
        const bool ph = pend.x != R(1) || pend.y != R(0);
        if (tsize >= 4 * kNT) {
            for (uint32_t j0 = 0; j0 < tsize; j0 += 4 * kNT) {
                T v[4], w[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t li = swz_tid ^ swz<R>(j0 + u * kNT);
                    v[u] = tp[li];
                    w[u] = tf[li];
                    if (ph) {
                        v[u] = cmul(pend, v[u]);
                        w[u] = cmul(pend, w[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint64_t gi = base | dep_tid | ta.dep_hi[(j0 >> 8) + u];
                    psi[gi] = v[u];
                    phi[gi] = w[u];
                }
            }
        } else {
            for (uint32_t j = 0; j < tsize; j += kNT)
                if (j + tid < tsize) {
                    const uint64_t gi = base | dep_tid | ta.dep_hi[j >> 8];
                    const uint32_t li = swz_tid ^ swz<R>(j);
                    T v = tp[li], w = tf[li];
                    if (ph) {
                        v = cmul(pend, v);
                        w = cmul(pend, w);
                    }
                    psi[gi] = v;
                    phi[gi] = w;
                }
        }
        __syncthreads();
    }
    __syncthreads();
    const size_t nb = (size_t)gridDim.x * kAdjWaves;
    for (int oi = 0; oi < ta.n_ops && tid < (uint32_t)kAdjWaves; ++oi) {
        const AdjOp &ao = ops[oi];
        if (ao.kind == ADJ_ROT) {
            for (int j = 0; j < ao.nsub; ++j)
                partial[(size_t)ao.gslot[j] * nb + (size_t)blockIdx.x * kAdjWaves + tid] =
                    acc[ao.lslot[j] * kAdjWaves + tid];
        } else if (ao.kind == ADJ_BLOCK) {
            for (int j = 0; j < ao.nsub; ++j) {
                const AdjSub &u = subs[ao.sub0 + j];
                if (u.kind == SUB_ROT)
                    partial[(size_t)u.gslot * nb + (size_t)blockIdx.x * kAdjWaves + tid] =
                        acc[u.lslot * kAdjWaves + tid];
            }
        }
    }
}

template <typename R, int KM>
static int adj_grid_t(int m) {
    const size_t lds = adjoint_tile_lds(sizeof(R) == 8 ? 0 : 1, m);
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute((const void *)k_adj_tile<R, KM>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_adj_tile<R, KM>, kNT, lds) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per * cus;
}

int adjoint_tile_grid(int dtype, int m, int mfma_k) {
    if (dtype == 0)
        return mfma_k == 0 ? adj_grid_t<double, 0>(m)
               : mfma_k <= 3 ? adj_grid_t<double, 3>(m) : adj_grid_t<double, 5>(m);
    return mfma_k == 0 ? adj_grid_t<float, 0>(m)
           : mfma_k <= 3 ? adj_grid_t<float, 3>(m) : adj_grid_t<float, 5>(m);
}

template <typename R, int KM>
static hipError_t adj_tile_t(void *psi, void *phi, const TileArgs &ta, const AdjOp *ops,
                             const AdjSub *subs, const void *pool, int nrot, double *partial,
                             int grid, hipStream_t s) {
    using T = typename VT<R>::T;
    const size_t lds = adjoint_tile_lds(sizeof(R) == 8 ? 0 : 1, ta.m);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_adj_tile<R, KM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_adj_tile<R, KM>), dim3((unsigned)grid), dim3(kNT), lds, s, (T *)psi,
                       (T *)phi, ta, ops, subs, (const T *)pool, nrot, partial);
    return hipGetLastError();
}

template <typename R>
static hipError_t adj_tile_k(void *psi, void *phi, const TileArgs &ta, const AdjOp *ops,
                             const AdjSub *subs, const void *pool, int nrot, double *partial,
                             int grid, hipStream_t s) {
    if (ta.mfma_k == 0)
        return adj_tile_t<R, 0>(psi, phi, ta, ops, subs, pool, nrot, partial, grid, s);
    if (ta.mfma_k <= 3)
        return adj_tile_t<R, 3>(psi, phi, ta, ops, subs, pool, nrot, partial, grid, s);
    return adj_tile_t<R, 5>(psi, phi, ta, ops, subs, pool, nrot, partial, grid, s);
}

hipError_t adjoint_tile_pass(int dtype, void *psi, void *phi, const TileArgs &ta,
                             const AdjOp *ops, const AdjSub *subs, const void *pool, int nrot,
                             double *partial, int grid, hipStream_t s) {
    if (grid < 1 || nrot < 0 || nrot > kAdjMaxRot || ta.m < 1 ||
        ta.m > (dtype == 0 ? 12 : 13) || ta.mfma_k < 0 || ta.mfma_k > 5)
        return hipErrorInvalidValue;
    return dtype == 0
               ? adj_tile_k<double>(psi, phi, ta, ops, subs, pool, nrot, partial, grid, s)
               : adj_tile_k<float>(psi, phi, ta, ops, subs, pool, nrot, partial, grid, s);
}

}  // namespace dev
}  // namespace qsv
