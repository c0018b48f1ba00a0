// Batched expectation values: many small circuits, each with its own Pauli
// sum.  k_batch is a persistent launch: every workgroup repeatedly takes the
// next circuit from an atomic counter (circuits are ordered longest first),
// simulates it alone and writes <H>.  A state of at most MB qubits lives in
// LDS for its whole life; a larger one given to k_batch lives in a
// per-workgroup slot of global memory and is updated by LDS-tile passes
// planned on the host.  No workgroup ever waits for another, so the grid
// drains as soon as the counter passes the number of circuits.  The
// pass-major kernels further down serve the larger circuits otherwise.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "lds_ops.hpp"

namespace qsv {
namespace dev {

// tile positions of a state held whole in LDS: local bit i is qubit i
__constant__ uint32_t kIdentityPos[40] = {0,  1,  2,  3,  4,  5,  6,  7,  8,  9,  10, 11, 12, 13,
                                          14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27,
                                          28, 29, 30, 31, 32, 33, 34, 35, 36, 37, 38, 39};

template <typename R>
__device__ __forceinline__ double block_sum_b(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

// sum_t c_t Re(i^{ny_t} sum_j conj(psi_{j^x}) psi_j (-1)^{popcount(j & z)}),
// this thread's share, state `st` of 2^n amplitudes (LDS or global).  The
// sweeps issue the loads of U indices (U pairs) per thread before using any,
// so enough reads are in flight for a state in global memory; a tail loop
// takes the indices left over.
// Indices [lo, hi) only (lo, hi multiples of 2): for a string with X letters
// the pairs (j, j ^ x) whose lower member has pair index in [lo/2, hi/2), so
// chunks that split [0, 2^n) split every term's sum.
template <typename R, bool SWZ>
__device__ __forceinline__ double pauli_partial(const typename VT<R>::T *st, int n,
                                                const BatchTerm *__restrict__ terms, int nt,
                                                uint64_t lo, uint64_t hi) {
    using T = typename VT<R>::T;
    constexpr int U = sizeof(R) == 4 ? 8 : 4;
    double acc = 0.0;
    (void)n;
    const uint64_t bd = blockDim.x;
    auto at = [&](uint64_t j) -> T { return st[SWZ ? swz<R>((uint32_t)j) : j]; };
    for (int t = 0; t < nt; ++t) {
        const BatchTerm tm = terms[t];
        double sr = 0.0, si = 0.0;
        if (tm.x == 0) {
            auto add = [&](uint64_t j, const T &a) {
                const double p = (double)a.x * a.x + (double)a.y * a.y;
                sr += (__popcll(j & tm.z) & 1) ? -p : p;
            };
            uint64_t j = lo + threadIdx.x;
            for (; j + (U - 1) * bd < hi; j += U * bd) {
                T a[U];
#pragma unroll
                for (int u = 0; u < U; ++u) a[u] = at(j + u * bd);
#pragma unroll
                for (int u = 0; u < U; ++u) add(j + u * bd, a[u]);
            }
            for (; j < hi; j += bd) add(j, at(j));
        } else {
            const int h = 63 - __builtin_clzll(tm.x);
            const uint64_t lowm = (1ull << h) - 1;
            auto idx = [&](uint64_t g) { return ((g & ~lowm) << 1) | (g & lowm); };
            auto add = [&](uint64_t j, const T &a, const T &b) {
                const uint64_t j2 = j ^ tm.x;
                const double u = (double)b.x * a.x + (double)b.y * a.y;
                const double v = (double)b.x * a.y - (double)b.y * a.x;
                const double s1 = (__popcll(j & tm.z) & 1) ? -1.0 : 1.0;
                const double s2 = (__popcll(j2 & tm.z) & 1) ? -1.0 : 1.0;
                sr += (s1 + s2) * u;
                si += (s1 - s2) * v;
            };
            const uint64_t half = hi >> 1;
            uint64_t g = (lo >> 1) + threadIdx.x;
            for (; g + (U - 1) * bd < half; g += U * bd) {
                T a[U], b[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t j = idx(g + u * bd);
                    a[u] = at(j);
                    b[u] = at(j ^ tm.x);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) add(idx(g + u * bd), a[u], b[u]);
            }
            for (; g < half; g += bd) {
                const uint64_t j = idx(g);
                add(j, at(j), at(j ^ tm.x));
            }
        }
        // Re(i^{ny} (sr + i si))
        double re;
        switch (tm.ny & 3) {
        case 0: re = sr; break;
        case 1: re = -si; break;
        case 2: re = -sr; break;
        default: re = si; break;
        }
        acc += tm.c * re;
    }
    return acc;
}

// One tile t of a pass over a state in global memory (`slot`): load it (from
// |0...0> on the circuit's first pass), apply the pass's ops in LDS, store
// it.  The whole workgroup calls it; it ends with a barrier.
template <typename R, int KM>
__device__ __forceinline__ void batch_tile(typename VT<R>::T *tile, typename VT<R>::T *slot,
                                           const BatchPass &bp, uint64_t t, bool init,
                                           const TileOp *__restrict__ ops,
                                           const typename VT<R>::T *__restrict__ pool) {
    using T = typename VT<R>::T;
    const uint32_t tid = threadIdx.x;
    const int m = bp.m;
    const uint32_t *tpos = bp.tpos;
    const uint32_t tsize = 1u << m;
    // loads in flight per thread while a tile comes in or goes out
    constexpr int LD = sizeof(R) == 4 ? 8 : 4;
    // thread part of local index j0 + tid (used when tsize >= LD kNT)
    const uint64_t dep_tid = deposit_bits(tid, tpos, m < 8 ? m : 8);
    const uint32_t swz_tid = swz<R>(tid);
    uint64_t base = t;
    for (int i = 0; i < m; ++i) {
        const uint64_t lowm = (1ull << tpos[i]) - 1;
        base = ((base & ~lowm) << 1) | (base & lowm);
    }
    // loads go out LD at a time, before their LDS writes (tiles of at least
    // LD * kNT amplitudes; smaller ones one at a time)
    if (tsize < LD * kNT) {
        for (uint32_t l = tid; l < tsize; l += kNT) {
            const uint64_t gi = base | deposit_bits(l, tpos, m);
            T v;
            if (init) {
                v.x = (gi == 0) ? R(1) : R(0);
                v.y = R(0);
            } else {
                v = slot[gi];
            }
            tile[swz<R>(l)] = v;
        }
    } else for (uint32_t j0 = 0; j0 < tsize; j0 += LD * kNT) {
        T v[LD];
#pragma unroll
        for (int u = 0; u < LD; ++u) {
            const uint64_t gi = base | dep_tid | deposit_bits(j0 + u * kNT, tpos, m);
            if (init) {
                v[u].x = (gi == 0) ? R(1) : R(0);
                v[u].y = R(0);
            } else {
                v[u] = slot[gi];
            }
        }
#pragma unroll
        for (int u = 0; u < LD; ++u) tile[swz_tid ^ swz<R>(j0 + u * kNT)] = v[u];
    }
    __syncthreads();
    for (int o = 0; o < bp.op_count; ++o) {
        lds_op<R, KM>(tile, m, base, tpos, ops[bp.op_begin + o], pool);
        __syncthreads();
    }
    if (tsize < LD * kNT) {
        for (uint32_t l = tid; l < tsize; l += kNT)
            slot[base | deposit_bits(l, tpos, m)] = tile[swz<R>(l)];
    } else for (uint32_t j0 = 0; j0 < tsize; j0 += LD * kNT) {
        T v[LD];
#pragma unroll
        for (int u = 0; u < LD; ++u) v[u] = tile[swz_tid ^ swz<R>(j0 + u * kNT)];
#pragma unroll
        for (int u = 0; u < LD; ++u)
            slot[base | dep_tid | deposit_bits(j0 + u * kNT, tpos, m)] = v[u];
    }
    __syncthreads();
}

template <typename R, int KM>
__global__ __launch_bounds__(kNT) void k_batch(const BatchCircuit *__restrict__ circuits,
                                               const int32_t *__restrict__ order, int count,
                                               const BatchPass *__restrict__ passes,
                                               const TileOp *__restrict__ ops,
                                               const typename VT<R>::T *__restrict__ pool,
                                               const BatchTerm *__restrict__ terms,
                                               typename VT<R>::T *__restrict__ scratch,
                                               uint64_t slot_amps, int mb,
                                               unsigned int *counter, double *out) {
    using T = typename VT<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);
    __shared__ int s_next;
    __shared__ double sh[16];
    T *slot = scratch + (uint64_t)blockIdx.x * slot_amps;
    const uint32_t tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_next = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int ci = s_next;
        __syncthreads();
        if (ci >= count) break;
        const BatchCircuit bc = circuits[order[ci]];
        const int n = bc.n;
        double part;
        if (n <= mb) {
            // whole state in LDS: |0...0>, every op of the single pass, <H>
            const uint32_t dim = 1u << n;
            for (uint32_t l = tid; l < dim; l += kNT) {
                T v;
                v.x = (l == 0) ? R(1) : R(0);
                v.y = R(0);
                tile[swz<R>(l)] = v;
            }
            __syncthreads();
            for (int p = 0; p < bc.pass_count; ++p) {
                const BatchPass &bp = passes[bc.pass_begin + p];
                for (int o = 0; o < bp.op_count; ++o) {
                    lds_op<R, KM>(tile, n, 0, kIdentityPos, ops[bp.op_begin + o], pool);
                    __syncthreads();
                }
            }
            part = pauli_partial<R, true>(tile, n, terms + bc.term_begin, bc.term_count, 0,
                                          1ull << n);
        } else {
            // state in this workgroup's global slot, updated by tile passes
            for (int p = 0; p < bc.pass_count; ++p) {
                const BatchPass &bp = passes[bc.pass_begin + p];
                const uint64_t ntiles = 1ull << (n - bp.m);
                for (uint64_t t = 0; t < ntiles; ++t)
                    batch_tile<R, KM>(tile, slot, bp, t, p == 0, ops, pool);
            }
            if (bc.pass_count == 0) {
                const uint64_t dim = 1ull << n;
                for (uint64_t j = tid; j < dim; j += kNT) {
                    T v;
                    v.x = (j == 0) ? R(1) : R(0);
                    v.y = R(0);
                    slot[j] = v;
                }
                __syncthreads();
            }
            part = pauli_partial<R, false>(slot, n, terms + bc.term_begin, bc.term_count, 0,
                                           1ull << n);
        }
        const double tot = block_sum_b<R>(part, sh);
        if (tid == 0) out[bc.out_index] = tot;
        __syncthreads();
    }
}

__global__ void k_reset_counter(unsigned int *counter) { *counter = 0u; }

// ------------------------------------------------------ pass-major circuits
// |0...0> in the states of the register-path circuits: the region zeroed,
// then amplitude 0 of each state set to 1.
template <typename R>
__global__ void k_batch_zero(typename VT<R>::T *p, uint64_t n) {
    using T = typename VT<R>::T;
    T z;
    z.x = R(0);
    z.y = R(0);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = z;
}
template <typename R>
__global__ void k_batch_one(typename VT<R>::T *states, const uint64_t *__restrict__ starts,
                            int count) {
    using T = typename VT<R>::T;
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= count) return;
    T o;
    o.x = R(1);
    o.y = R(0);
    states[starts[i]] = o;
}

// Segment of work item `it`: the last segment whose first item is <= it (the
// host orders a launch's segments by first item, the first one at 0).
__device__ __forceinline__ int find_seg(const BatchSeg *__restrict__ segs, int nseg,
                                        uint64_t it) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].first <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One pass index of every pass-major circuit: work item = (circuit, tile),
// taken by the workgroups in a fixed stride (no counter, no waiting).  The
// kernel boundary orders a circuit's passes.
template <typename R, int KM>
__global__ __launch_bounds__(kNT) void k_batch_pass(const BatchSeg *__restrict__ segs, int nseg,
                                                    uint64_t items,
                                                    const BatchPass *__restrict__ passes,
                                                    const TileOp *__restrict__ ops,
                                                    const typename VT<R>::T *__restrict__ pool,
                                                    typename VT<R>::T *__restrict__ states) {
    using T = typename VT<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);
    for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const BatchSeg sg = segs[find_seg(segs, nseg, it)];
        batch_tile<R, KM>(tile, states + sg.state_off, passes[sg.pass], it - sg.first,
                          sg.init != 0, ops, pool);
    }
}

// The Pauli sums of the pass-major circuits: work item = (circuit, chunk k of
// C = 2^cl indices, cl = min(chunk_log, n)); partial[item] = the chunk's
// share of sum_t c_t <P_t>.  The chunk is read into LDS once and serves
// every term.  A term with X letters pairs j with j ^ x; the pair is taken
// by the chunk of its member with bit h = 0 (h: the highest X bit): within
// the chunk when h < cl, else by the chunks whose index has bit h - cl clear,
// which read the partner chunk k ^ (x >> cl) from global memory.  So a term
// reads half a state from global memory instead of a whole one, and a
// string of Z letters none.
template <typename R>
__global__ __launch_bounds__(kNT) void k_batch_pauli(const BatchSeg *__restrict__ segs, int nseg,
                                                     uint64_t items,
                                                     const BatchCircuit *__restrict__ circuits,
                                                     const BatchTerm *__restrict__ terms,
                                                     const typename VT<R>::T *__restrict__ states,
                                                     int chunk_log, double *__restrict__ partial) {
    using T = typename VT<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *ch = reinterpret_cast<T *>(smem_raw);
    __shared__ double sh[16];
    constexpr int U = sizeof(R) == 4 ? 8 : 4;   // global reads in flight per thread
    const uint32_t tid = threadIdx.x;
    for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const BatchSeg sg = segs[find_seg(segs, nseg, it)];
        const BatchCircuit bc = circuits[sg.circuit];
        const int cl = chunk_log < bc.n ? chunk_log : bc.n;
        const uint32_t C = 1u << cl;
        const uint64_t k = it - sg.first;
        const uint64_t j0 = k << cl;
        const T *st = states + sg.state_off;
        {
            // U loads of a thread out together before their LDS writes
            uint32_t l = tid;
            for (; l + (U - 1) * kNT < C; l += U * kNT) {
                T v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = st[j0 + l + u * kNT];
#pragma unroll
                for (int u = 0; u < U; ++u) ch[l + u * kNT] = v[u];
            }
            for (; l < C; l += kNT) ch[l] = st[j0 + l];
        }
        __syncthreads();
        double acc = 0.0;
        for (int t = 0; t < bc.term_count; ++t) {
            const BatchTerm tm = terms[bc.term_begin + t];
            double sr = 0.0, si = 0.0;
            if (tm.x == 0) {
                for (uint32_t l = tid; l < C; l += kNT) {
                    const T a = ch[l];
                    const double p = (double)a.x * a.x + (double)a.y * a.y;
                    sr += (__popcll((j0 + l) & tm.z) & 1) ? -p : p;
                }
            } else {
                const int h = 63 - __builtin_clzll(tm.x);
                auto add = [&](uint64_t j, const T &a, const T &b) {
                    const uint64_t j2 = j ^ tm.x;
                    const double u = (double)b.x * a.x + (double)b.y * a.y;
                    const double v = (double)b.x * a.y - (double)b.y * a.x;
                    const double s1 = (__popcll(j & tm.z) & 1) ? -1.0 : 1.0;
                    const double s2 = (__popcll(j2 & tm.z) & 1) ? -1.0 : 1.0;
                    sr += (s1 + s2) * u;
                    si += (s1 - s2) * v;
                };
                if (h < cl) {
                    // both members in the chunk: pair g has local index g
                    // with a 0 inserted at bit h
                    const uint32_t lowm = (1u << h) - 1;
                    const uint32_t xl = (uint32_t)tm.x;
                    for (uint32_t g = tid; g < (C >> 1); g += kNT) {
                        const uint32_t l = ((g & ~lowm) << 1) | (g & lowm);
                        add(j0 + l, ch[l], ch[l ^ xl]);
                    }
                } else if (((j0 >> h) & 1) == 0) {
                    const T *pp = st + ((j0 ^ tm.x) & ~(uint64_t)(C - 1));
                    const uint32_t xl = (uint32_t)(tm.x & (C - 1));
                    uint32_t l = tid;
                    for (; l + (U - 1) * kNT < C; l += U * kNT) {
                        T b[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) b[u] = pp[(l + u * kNT) ^ xl];
#pragma unroll
                        for (int u = 0; u < U; ++u) add(j0 + l + u * kNT, ch[l + u * kNT], b[u]);
                    }
                    for (; l < C; l += kNT) add(j0 + l, ch[l], pp[l ^ xl]);
                }
            }
            // Re(i^{ny} (sr + i si))
            double re;
            switch (tm.ny & 3) {
            case 0: re = sr; break;
            case 1: re = -si; break;
            case 2: re = -sr; break;
            default: re = si; break;
            }
            acc += tm.c * re;
        }
        const double tot = block_sum_b<R>(acc, sh);
        if (tid == 0) partial[it] = tot;
        __syncthreads();   // the chunk and sh are rewritten by the next item
    }
}

// <H> of each pass-major circuit: its chunk sums added in chunk order (the
// same order on every run).
__global__ void k_batch_finish(const BatchSeg *__restrict__ segs, int nseg, uint64_t items,
                               const BatchCircuit *__restrict__ circuits,
                               const double *__restrict__ partial, double *__restrict__ out) {
    const int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= nseg) return;
    const uint64_t b = segs[s].first, e = s + 1 < nseg ? segs[s + 1].first : items;
    double acc = 0.0;
    for (uint64_t i = b; i < e; ++i) acc += partial[i];
    out[circuits[segs[s].circuit].out_index] = acc;
}

template <typename R, int KM>
static hipError_t batch_t(const BatchLaunch &L, hipStream_t s) {
    using T = typename VT<R>::T;
    const size_t lds = sizeof(T) << L.mb;
    static size_t attr = 0;
    if (attr < lds) {
        hipError_t e = hipFuncSetAttribute((const void *)k_batch<R, KM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = lds;
    }
    if (L.count > 0) {
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, L.counter);
        hipLaunchKernelGGL((k_batch<R, KM>), dim3(L.grid), dim3(kNT), lds, s, L.circuits,
                           L.order, L.count, L.passes, L.ops, (const T *)L.pool, L.terms,
                           (T *)L.scratch, L.slot_amps, L.mb, L.counter, L.out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!L.pass_major) return hipSuccess;
    if (L.n_reg_launches > 0) {
        T *rs = (T *)L.states + L.reg_state_off;
        const unsigned zg = (unsigned)std::min<uint64_t>((L.reg_amps + 255) / 256, 65536);
        hipLaunchKernelGGL((k_batch_zero<R>), dim3(zg), dim3(256), 0, s, rs, L.reg_amps);
        hipLaunchKernelGGL((k_batch_one<R>), dim3((L.n_reg_states + 255) / 256), dim3(256), 0, s,
                           (T *)L.states, L.reg_starts, L.n_reg_states);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        for (int i = 0; i < L.n_reg_launches; ++i) {
            const int sb = L.reg_seg_begin[i], ns = L.reg_seg_begin[i + 1] - sb;
            e = launch_tile_reg_batch(sizeof(R) == 8 ? 0 : 1, L.reg_dg[i] != 0, L.states,
                                      L.reg_segs + sb, ns, L.reg_items[i], L.tas, L.rops,
                                      L.reg_pool, L.reg_img_max, s);
            if (e != hipSuccess) return e;
        }
    }
    static size_t attr_p = 0;
    if (attr_p < lds) {
        hipError_t e = hipFuncSetAttribute((const void *)k_batch_pass<R, KM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_p = lds;
    }
    for (int i = 0; i <= L.n_pass_launches; ++i) {
        const int sb = L.seg_begin[i], ns = L.seg_begin[i + 1] - sb;
        const uint64_t items = L.items[i];
        if (items == 0 || ns <= 0) continue;
        const unsigned grid = (unsigned)std::min<uint64_t>(items, L.grid_big);
        if (i < L.n_pass_launches) {
            hipLaunchKernelGGL((k_batch_pass<R, KM>), dim3(grid), dim3(kNT), lds, s, L.segs + sb,
                               ns, items, L.passes, L.ops, (const T *)L.pool, (T *)L.states);
        } else {
            const size_t chb = sizeof(T) << L.chunk_log;
            static size_t attr_c = 0;
            if (attr_c < chb) {
                hipError_t e = hipFuncSetAttribute((const void *)k_batch_pauli<R>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)chb);
                if (e != hipSuccess) return e;
                attr_c = chb;
            }
            hipLaunchKernelGGL((k_batch_pauli<R>), dim3(grid), dim3(kNT), chb, s, L.segs + sb, ns,
                               items, L.circuits, L.terms, (const T *)L.states, L.chunk_log,
                               L.partial);
            hipLaunchKernelGGL(k_batch_finish, dim3((ns + 255) / 256), dim3(256), 0, s,
                               L.segs + sb, ns, items, L.circuits, (const double *)L.partial,
                               L.out);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Kernel variant for the widest matrix-core op of the batch: up to 3 qubits
// (the autotuned fusion widths) or up to 5 (wider user gates).
hipError_t batch_launch(int dtype, const BatchLaunch &L, hipStream_t s) {
    if (L.mfma_k > 5) return hipErrorInvalidValue;
    if (dtype == 0)
        return L.mfma_k <= 3 ? batch_t<double, 3>(L, s) : batch_t<double, 5>(L, s);
    return L.mfma_k <= 3 ? batch_t<float, 3>(L, s) : batch_t<float, 5>(L, s);
}

template <typename R, int KM>
static int batch_occ_t(int mb) {
    using T = typename VT<R>::T;
    int blocks = 0;
    (void)hipFuncSetAttribute((const void *)k_batch<R, KM>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sizeof(T) << mb));
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &blocks, k_batch<R, KM>, kNT, sizeof(T) << mb);
    return e == hipSuccess ? blocks : 0;
}

template <typename R, int KM>
static int batch_pass_occ_t(int mb) {
    using T = typename VT<R>::T;
    int blocks = 0;
    (void)hipFuncSetAttribute((const void *)k_batch_pass<R, KM>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sizeof(T) << mb));
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &blocks, k_batch_pass<R, KM>, kNT, sizeof(T) << mb);
    return e == hipSuccess ? blocks : 0;
}

int batch_pass_occupancy(int dtype, int mb, int mfma_k) {
    if (dtype == 0)
        return mfma_k <= 3 ? batch_pass_occ_t<double, 3>(mb) : batch_pass_occ_t<double, 5>(mb);
    return mfma_k <= 3 ? batch_pass_occ_t<float, 3>(mb) : batch_pass_occ_t<float, 5>(mb);
}

int batch_occupancy(int dtype, int mb, int mfma_k) {
    if (dtype == 0) return mfma_k <= 3 ? batch_occ_t<double, 3>(mb) : batch_occ_t<double, 5>(mb);
    return mfma_k <= 3 ? batch_occ_t<float, 3>(mb) : batch_occ_t<float, 5>(mb);
}

}  // namespace dev
}  // namespace qsv
