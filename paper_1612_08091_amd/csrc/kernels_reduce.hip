// Reductions and whole-state operations: probabilities, masked probability
// sums, Pauli-sum expectation values, sampling, collapse after measurement,
// qubit allocation (zero extension) and deallocation (compaction).  Every sum
// is accumulated in double precision whatever the state's dtype.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "device.hpp"

namespace qsv {
namespace dev {

template <typename R> struct V2r;
template <> struct V2r<double> { using T = double2; };
template <> struct V2r<float> { using T = float2; };

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum over the block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (w == 0) {
        v = (lane < (int)(blockDim.x >> 6)) ? sh[lane] : 0.0;
        v = wave_sum(v);
    }
    return v;
}

__device__ __forceinline__ uint64_t expand_idx(uint64_t g, const IndexArgs &ia) {
    for (int i = 0; i < ia.npos; ++i) {
        const uint64_t lowm = (1ull << ia.pos[i]) - 1;
        g = ((g & ~lowm) << 1) | (g & lowm);
    }
    return g | ia.ones;
}

static unsigned red_grid(uint64_t work) {
    uint64_t b = (work + kRedThreads - 1) / kRedThreads;
    if (b > kRedBlocks) b = kRedBlocks;
    if (b == 0) b = 1;
    return (unsigned)b;
}

// ------------------------------------------------------------ probability
template <typename R>
__global__ __launch_bounds__(kRedThreads) void k_prob_masked(const typename V2r<R>::T *psi,
                                                             uint64_t ngroups, IndexArgs ia,
                                                             double *partial) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const auto a = psi[expand_idx(g, ia)];
        const double re = a.x, im = a.y;
        acc += re * re + im * im;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

template <typename R>
__global__ __launch_bounds__(kRedThreads) void k_prob_split(const typename V2r<R>::T *psi,
                                                            uint64_t dim, int q,
                                                            double *partial) {
    __shared__ double sh[16];
    double a0 = 0.0, a1 = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const auto a = psi[i];
        const double p = (double)a.x * a.x + (double)a.y * a.y;
        if ((i >> q) & 1) a1 += p;
        else a0 += p;
    }
    a0 = block_sum(a0, sh);
    a1 = block_sum(a1, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = a0;
        partial[2 * blockIdx.x + 1] = a1;
    }
}

// out[j] = sum_b partial[b * stride + j] for j < width
__global__ __launch_bounds__(kRedThreads) void k_finish(const double *partial, int nblocks,
                                                        int stride, int width, double *out) {
    __shared__ double sh[16];
    for (int j = 0; j < width; ++j) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += partial[b * stride + j];
        acc = block_sum(acc, sh);
        if (threadIdx.x == 0) out[j] = acc;
    }
}

size_t reduce_workspace_bytes(int) { return sizeof(double) * 2 * kRedBlocks; }

// --------------------------------------------------- allocation-free form
// Partial sums of prob_masked_noalloc: one per block of k_prob_masked (at most
// kRedBlocks).  Every GPU holds its own copy until the process ends; each call
// writes the slots it reads, so nothing needs clearing, and calls that overlap
// on one GPU race on it.
constexpr int kScratchDoubles = kRedBlocks;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's `scratch` (resolved once per device, with the
// device current; host code never uses the array's own name).
hipError_t scratch_ptr(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

int prob_noalloc_partials(uint64_t ngroups) { return (int)red_grid(ngroups); }
int prob_noalloc_capacity() { return kScratchDoubles; }

hipError_t prob_masked_noalloc(int dtype, const void *psi, uint64_t ngroups, const IndexArgs &ia,
                               double *out_dev, hipStream_t s) {
    if ((int)red_grid(ngroups) > kScratchDoubles) return hipErrorInvalidValue;
    double *ws = nullptr;
    const hipError_t e = scratch_ptr(&ws);
    if (e != hipSuccess) return e;
    return prob_masked(dtype, psi, ngroups, ia, ws, out_dev, s);
}

hipError_t prob_masked(int dtype, const void *psi, uint64_t ngroups, const IndexArgs &ia,
                       double *ws, double *out_dev, hipStream_t s) {
    const unsigned g = red_grid(ngroups);
    if (dtype == 0)
        hipLaunchKernelGGL(k_prob_masked<double>, dim3(g), dim3(kRedThreads), 0, s,
                           (const double2 *)psi, ngroups, ia, ws);
    else
        hipLaunchKernelGGL(k_prob_masked<float>, dim3(g), dim3(kRedThreads), 0, s,
                           (const float2 *)psi, ngroups, ia, ws);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, s, ws, (int)g, 1, 1, out_dev);
    return hipGetLastError();
}

hipError_t prob_split(int dtype, const void *psi, int nq, int q, double *ws, double *out_dev,
                      hipStream_t s) {
    const uint64_t dim = 1ull << nq;
    const unsigned g = red_grid(dim);
    if (dtype == 0)
        hipLaunchKernelGGL(k_prob_split<double>, dim3(g), dim3(kRedThreads), 0, s,
                           (const double2 *)psi, dim, q, ws);
    else
        hipLaunchKernelGGL(k_prob_split<float>, dim3(g), dim3(kRedThreads), 0, s,
                           (const float2 *)psi, dim, q, ws);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, s, ws, (int)g, 2, 2, out_dev);
    return hipGetLastError();
}

// ------------------------------------------------ reduced density matrix
// rho_T[a][b] = sum over the other bits of psi[i_a] conj(psi[i_b]), where i_a
// is the index whose target bits (positions ia.pos, ascending, and tp[j] the
// position of target j) take the bits of a.  Each block writes its partial
// 2^K x 2^K complex matrix (2 * 4^K doubles, row-major, re/im) to
// partial[block * 2 * 4^K ...].
template <typename R, int K>
__global__ __launch_bounds__(kRedThreads) void k_reduced_dm(const typename V2r<R>::T *psi,
                                                            uint64_t ngroups, IndexArgs ia,
                                                            int tp0, int tp1, double *partial) {
    constexpr int D = 1 << K;
    __shared__ double sh[16];
    double re[D][D], im[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) re[a][b] = im[a][b] = 0.0;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t base = expand_idx(g, ia);
        double xr[D], xi[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            uint64_t i = base;
            if (a & 1) i |= 1ull << tp0;
            if (K > 1 && (a & 2)) i |= 1ull << tp1;
            const auto v = psi[i];
            xr[a] = v.x;
            xi[a] = v.y;
        }
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) {
                re[a][b] += xr[a] * xr[b] + xi[a] * xi[b];
                im[a][b] += xi[a] * xr[b] - xr[a] * xi[b];
            }
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            const double sr = block_sum(re[a][b], sh);
            const double si = block_sum(im[a][b], sh);
            if (threadIdx.x == 0) {
                partial[(size_t)blockIdx.x * 2 * D * D + 2 * (a * D + b)] = sr;
                partial[(size_t)blockIdx.x * 2 * D * D + 2 * (a * D + b) + 1] = si;
            }
        }
}

size_t reduced_dm_workspace_bytes() { return sizeof(double) * 2 * 16 * kRedBlocks; }

hipError_t reduced_dm(int dtype, const void *psi, int nq, int k, const int *pos, double *ws,
                      double *out_dev, hipStream_t s) {
    if (k < 1 || k > 2 || nq < k) return hipErrorInvalidValue;
    IndexArgs ia;
    int sorted[2] = {pos[0], k > 1 ? pos[1] : 0};
    if (k > 1 && sorted[1] < sorted[0]) std::swap(sorted[0], sorted[1]);
    ia.npos = k;
    for (int j = 0; j < k; ++j) ia.pos[j] = (uint8_t)sorted[j];
    const uint64_t ngroups = 1ull << (nq - k);
    const unsigned g = red_grid(ngroups);
    const int w = 2 << (2 * k);
    const int tp1 = k > 1 ? pos[1] : 0;
#define QSV_RDM(R, K)                                                                        \
    hipLaunchKernelGGL((k_reduced_dm<R, K>), dim3(g), dim3(kRedThreads), 0, s,               \
                       (const typename V2r<R>::T *)psi, ngroups, ia, pos[0], tp1, ws)
    if (dtype == 0) {
        if (k == 1) QSV_RDM(double, 1);
        else QSV_RDM(double, 2);
    } else {
        if (k == 1) QSV_RDM(float, 1);
        else QSV_RDM(float, 2);
    }
#undef QSV_RDM
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedThreads), 0, s, ws, (int)g, w, w, out_dev);
    return hipGetLastError();
}

template <typename R>
__global__ void k_probs(const typename V2r<R>::T *psi, uint64_t dim, double *out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const auto a = psi[i];
        out[i] = (double)a.x * a.x + (double)a.y * a.y;
    }
}

hipError_t probs(int dtype, const void *psi, uint64_t dim, double *out_dev, hipStream_t s) {
    const unsigned g = (unsigned)std::min<uint64_t>((dim + 255) / 256, 1ull << 20);
    if (dtype == 0)
        hipLaunchKernelGGL(k_probs<double>, dim3(g), dim3(256), 0, s, (const double2 *)psi, dim,
                           out_dev);
    else
        hipLaunchKernelGGL(k_probs<float>, dim3(g), dim3(256), 0, s, (const float2 *)psi, dim,
                           out_dev);
    return hipGetLastError();
}

// ------------------------------------------------------------ Pauli sums
// <P> for P with x mask x and z mask z equals i^{n_Y} sum_j conj(psi_{j^x})
// psi_j (-1)^{popcount(j & z)}.  Terms sharing x are evaluated together; a
// pair (j, j^x) is read once.  Chunk c holds up to 8 terms with one x mask.
constexpr int kPauliChunk = 8;
constexpr int kPauliBlocks = 512;

struct PauliChunk {
    uint64_t x;
    int32_t hbit;    // highest set bit of x, -1 for x == 0
    int32_t nt;
    int32_t term[kPauliChunk];
};

template <typename R>
__global__ __launch_bounds__(kRedThreads) void k_pauli(const typename V2r<R>::T *psi, int nq,
                                                       const PauliChunk *chunks,
                                                       const uint64_t *zmask, double *partial) {
    __shared__ double sh[16];
    const PauliChunk ch = chunks[blockIdx.y];
    uint64_t z[kPauliChunk];
#pragma unroll
    for (int t = 0; t < kPauliChunk; ++t) z[t] = (t < ch.nt) ? zmask[ch.term[t]] : 0;
    double ar[kPauliChunk], ai[kPauliChunk];
#pragma unroll
    for (int t = 0; t < kPauliChunk; ++t) ar[t] = ai[t] = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    if (ch.hbit < 0) {
        const uint64_t dim = 1ull << nq;
        for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < dim; j += stride) {
            const auto a = psi[j];
            const double p = (double)a.x * a.x + (double)a.y * a.y;
#pragma unroll
            for (int t = 0; t < kPauliChunk; ++t)
                ar[t] += (__popcll(j & z[t]) & 1) ? -p : p;
        }
    } else {
        const uint64_t npairs = 1ull << (nq - 1);
        const uint64_t lowm = (1ull << ch.hbit) - 1;
        for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < npairs;
             g += stride) {
            const uint64_t j = ((g & ~lowm) << 1) | (g & lowm);
            const uint64_t j2 = j ^ ch.x;
            const auto a = psi[j];
            const auto b = psi[j2];
            // w = conj(b) * a
            const double u = (double)b.x * a.x + (double)b.y * a.y;
            const double v = (double)b.x * a.y - (double)b.y * a.x;
#pragma unroll
            for (int t = 0; t < kPauliChunk; ++t) {
                const double s1 = (__popcll(j & z[t]) & 1) ? -1.0 : 1.0;
                const double s2 = (__popcll(j2 & z[t]) & 1) ? -1.0 : 1.0;
                ar[t] += (s1 + s2) * u;
                ai[t] += (s1 - s2) * v;
            }
        }
    }
    double *out = partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2 * kPauliChunk;
#pragma unroll
    for (int t = 0; t < kPauliChunk; ++t) {
        const double r = block_sum(ar[t], sh);
        const double i = block_sum(ai[t], sh);
        if (threadIdx.x == 0) {
            out[2 * t] = r;
            out[2 * t + 1] = i;
        }
    }
}

// Combine: out = sum_chunks sum_t coef[term] * i^{ny[term]} * sum_blocks partial.
__global__ __launch_bounds__(kRedThreads) void k_pauli_finish(const double *partial,
                                                              int nchunks, int nblocks,
                                                              const PauliChunk *chunks,
                                                              const double *coef,
                                                              const int32_t *ny, double *out) {
    __shared__ double sh[16];
    double tr = 0.0, ti = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        const PauliChunk ch = chunks[c];
        for (int t = 0; t < ch.nt; ++t) {
            double sr = 0.0, si = 0.0;
            for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
                const double *p = partial + ((size_t)c * nblocks + b) * 2 * kPauliChunk;
                sr += p[2 * t];
                si += p[2 * t + 1];
            }
            sr = block_sum(sr, sh);
            si = block_sum(si, sh);
            if (threadIdx.x == 0) {
                const int term = ch.term[t];
                double vr = sr, vi = si;   // multiply by i^{ny}
                switch (ny[term] & 3) {
                case 1: { double tmp = vr; vr = -vi; vi = tmp; } break;
                case 2: vr = -vr; vi = -vi; break;
                case 3: { double tmp = vr; vr = vi; vi = -tmp; } break;
                default: break;
                }
                tr += coef[term] * vr;
                ti += coef[term] * vi;
            }
        }
    }
    if (threadIdx.x == 0) {
        out[0] = tr;
        out[1] = ti;
    }
}

// A Pauli sum whose X letters all lie on few qubits, in one read of the
// state: a workgroup takes tiles of 2^m amplitudes whose positions hold every
// qubit with an X letter (and the lowest positions, for contiguous reads),
// reads each tile into LDS once and forms every term's share from it: both
// members of each pair (j, j ^ x) lie in the tile.  Signs split into the part
// from the tile's base index and the part from the local index.  Per-thread
// sums over all tiles, then one block sum per term, the blocks added in order
// by k_pauli_tiled_finish.
constexpr int kPauliTiledTerms = 16;
// bit i of l placed at position tpos[i], i < m
__device__ __forceinline__ uint64_t pdeposit(uint32_t l, const uint32_t *tpos, int m) {
    uint64_t out = 0;
    for (int i = 0; i < m; ++i) out |= (uint64_t)((l >> i) & 1u) << tpos[i];
    return out;
}
struct PauliTiled {
    int32_t m, nt;
    uint32_t tpos[16];                 // tile positions, ascending
    uint32_t xl[kPauliTiledTerms];     // X mask on local bits
    uint32_t zl[kPauliTiledTerms];     // Z mask on local bits
    uint64_t zo[kPauliTiledTerms];     // Z mask outside the tile
    int32_t hb[kPauliTiledTerms];      // highest bit of xl, -1 for none
    uint32_t zterms;                   // bit t: term t has no X letter
};

template <typename R>
__global__ __launch_bounds__(kRedThreads) void k_pauli_tiled(const typename V2r<R>::T *psi, int nq,
                                                             const PauliTiled pt,
                                                             double *partial) {
    using T = typename V2r<R>::T;
    // tiles of 2^m amplitudes, m = 11 (complex128) or 12 (complex64): 2^m /
    // 256 loads per thread
    constexpr int KL = sizeof(R) == 8 ? 8 : 16;
    extern __shared__ __align__(16) unsigned char smem_p[];
    T *ch = reinterpret_cast<T *>(smem_p);
    __shared__ double sh[16];
    const uint32_t tid = threadIdx.x;
    const uint32_t tsize = 1u << pt.m;
    const uint64_t ntiles = 1ull << (nq - pt.m);
    const uint64_t dep_tid = pdeposit(tid, pt.tpos, 8);
    double ar[kPauliTiledTerms], ai[kPauliTiledTerms];
#pragma unroll
    for (int t = 0; t < kPauliTiledTerms; ++t) ar[t] = ai[t] = 0.0;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        uint64_t base = tile;
        for (int i = 0; i < pt.m; ++i) {
            const uint64_t lowm = (1ull << pt.tpos[i]) - 1;
            base = ((base & ~lowm) << 1) | (base & lowm);
        }
        // local index tid + 256 k: the low 8 bits from the thread, the rest
        // uniform per k; all of a thread's loads go out before any LDS write
        T v[KL];
#pragma unroll
        for (int k = 0; k < KL; ++k) v[k] = psi[base | dep_tid | pdeposit((uint32_t)k << 8, pt.tpos, pt.m)];
#pragma unroll
        for (int k = 0; k < KL; ++k) ch[tid + ((uint32_t)k << 8)] = v[k];
        __syncthreads();
        // the strings of Z letters together, one read of the tile: sign bit
        // of term t = parity of (l & zl[t]) ^ bit t of sbits (the base part)
        if (pt.zterms) {
            uint32_t sbits = 0;
#pragma unroll
            for (int t = 0; t < kPauliTiledTerms; ++t)
                if ((pt.zterms >> t) & 1u) sbits |= (uint32_t)(__popcll(base & pt.zo[t]) & 1) << t;
            for (uint32_t l = tid; l < tsize; l += kRedThreads) {
                const T a = ch[l];
                const double p = (double)a.x * a.x + (double)a.y * a.y;
#pragma unroll
                for (int t = 0; t < kPauliTiledTerms; ++t)
                    if ((pt.zterms >> t) & 1u)
                        ar[t] += ((__popc(l & pt.zl[t]) ^ (sbits >> t)) & 1) ? -p : p;
            }
        }
#pragma unroll
        for (int t = 0; t < kPauliTiledTerms; ++t) {
            if (t >= pt.nt || pt.hb[t] < 0) continue;
            const double sb = (__popcll(base & pt.zo[t]) & 1) ? -1.0 : 1.0;
            const uint32_t zl = pt.zl[t];
            {
                const uint32_t xl = pt.xl[t];
                const uint32_t lowm = (1u << pt.hb[t]) - 1;
                double sr = 0.0, si = 0.0;
                for (uint32_t g = tid; g < (tsize >> 1); g += kRedThreads) {
                    const uint32_t l = ((g & ~lowm) << 1) | (g & lowm);
                    const uint32_t l2 = l ^ xl;
                    const T a = ch[l], b = ch[l2];
                    const double u = (double)b.x * a.x + (double)b.y * a.y;
                    const double v = (double)b.x * a.y - (double)b.y * a.x;
                    const double s1 = (__popc(l & zl) & 1) ? -1.0 : 1.0;
                    const double s2 = (__popc(l2 & zl) & 1) ? -1.0 : 1.0;
                    sr += (s1 + s2) * u;
                    si += (s1 - s2) * v;
                }
                ar[t] += sb * sr;
                ai[t] += sb * si;
            }
        }
        __syncthreads();   // the tile is rewritten next
    }
    double *out = partial + (size_t)blockIdx.x * 2 * kPauliTiledTerms;
#pragma unroll
    for (int t = 0; t < kPauliTiledTerms; ++t) {
        if (t >= pt.nt) continue;
        const double r = block_sum(ar[t], sh);
        const double i = block_sum(ai[t], sh);
        if (tid == 0) {
            out[2 * t] = r;
            out[2 * t + 1] = i;
        }
    }
}

__global__ __launch_bounds__(kRedThreads) void k_pauli_tiled_finish(const double *partial,
                                                                    int nblocks, int nt,
                                                                    const double *coef,
                                                                    const int32_t *ny,
                                                                    double *out) {
    __shared__ double sh[16];
    double tr = 0.0, ti = 0.0;
    for (int t = 0; t < nt; ++t) {
        double sr = 0.0, si = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
            sr += partial[(size_t)b * 2 * kPauliTiledTerms + 2 * t];
            si += partial[(size_t)b * 2 * kPauliTiledTerms + 2 * t + 1];
        }
        sr = block_sum(sr, sh);
        si = block_sum(si, sh);
        if (threadIdx.x == 0) {
            double vr = sr, vi = si;   // multiply by i^{ny}
            switch (ny[t] & 3) {
            case 1: { double tmp = vr; vr = -vi; vi = tmp; } break;
            case 2: vr = -vr; vi = -vi; break;
            case 3: { double tmp = vr; vr = vi; vi = -tmp; } break;
            default: break;
            }
            tr += coef[t] * vr;
            ti += coef[t] * vi;
        }
    }
    if (threadIdx.x == 0) {
        out[0] = tr;
        out[1] = ti;
    }
}

constexpr int kPauliTiledBlocks = 2048;

size_t pauli_workspace_bytes(int, int nchunks, int) {
    const size_t chunked = sizeof(double) * 2 * kPauliChunk * (size_t)kPauliBlocks * nchunks +
                           sizeof(PauliChunk) * nchunks + 256;
    const size_t tiled = sizeof(double) * 2 * kPauliTiledTerms * (size_t)kPauliTiledBlocks + 256;
    return chunked > tiled ? chunked : tiled;
}

// The tiled plan when every term's X letters fit in a tile of m bits (with
// the lowest positions filling the rest) and there are at most 16 terms:
// then one read of the state serves the whole sum.
static bool pauli_tiled_plan(int dtype, int nq, int ngroups, const PauliGroup *groups,
                             const uint64_t *z_host, int nterms, PauliTiled &pt) {
    const int m = dtype == 0 ? 11 : 12;   // 32 KiB of LDS (the kernel assumes these sizes)
    if (z_host == nullptr || nterms < 1 || nterms > kPauliTiledTerms || nq < m + 1) return false;
    uint64_t u = 0;
    for (int g = 0; g < ngroups; ++g) u |= groups[g].x;
    if (__builtin_popcountll(u) > m - 3) return false;
    uint64_t tile = u;
    for (int b = 0; b < nq && __builtin_popcountll(tile) < m; ++b) tile |= 1ull << b;
    pt = PauliTiled{};
    pt.m = m;
    pt.nt = nterms;
    int loc[64];
    int c = 0;
    for (int b = 0; b < 64; ++b) {
        loc[b] = -1;
        if ((tile >> b) & 1) {
            loc[b] = c;
            pt.tpos[c++] = (uint32_t)b;
        }
    }
    auto to_local = [&](uint64_t mask) {
        uint32_t r = 0;
        for (int b = 0; b < 64; ++b)
            if (((mask >> b) & 1) && loc[b] >= 0) r |= 1u << loc[b];
        return r;
    };
    for (int g = 0; g < ngroups; ++g)
        for (int k = 0; k < groups[g].count; ++k) {
            const int t = groups[g].first + k;
            pt.xl[t] = to_local(groups[g].x);
            pt.zl[t] = to_local(z_host[t]);
            pt.zo[t] = z_host[t] & ~tile;
            pt.hb[t] = pt.xl[t] ? 31 - __builtin_clz(pt.xl[t]) : -1;
            if (pt.hb[t] < 0) pt.zterms |= 1u << t;
        }
    return true;
}

hipError_t pauli_expectation(int dtype, const void *psi, int nq, int ngroups,
                             const PauliGroup *groups, const uint64_t *z_dev,
                             const double *coef_dev, const int32_t *ny_dev, int nterms,
                             double *ws, size_t ws_bytes, double *out_dev, hipStream_t s,
                             const uint64_t *z_host) {
    PauliTiled pt;
    if (pauli_tiled_plan(dtype, nq, ngroups, groups, z_host, nterms, pt)) {
        const uint64_t ntiles = 1ull << (nq - pt.m);
        const unsigned nb = (unsigned)(ntiles < kPauliTiledBlocks ? ntiles : kPauliTiledBlocks);
        if (sizeof(double) * 2 * kPauliTiledTerms * nb > ws_bytes) return hipErrorInvalidValue;
        const size_t lds = (dtype == 0 ? 16 : 8) << pt.m;
        if (dtype == 0)
            hipLaunchKernelGGL(k_pauli_tiled<double>, dim3(nb), dim3(kRedThreads), lds, s,
                               (const double2 *)psi, nq, pt, ws);
        else
            hipLaunchKernelGGL(k_pauli_tiled<float>, dim3(nb), dim3(kRedThreads), lds, s,
                               (const float2 *)psi, nq, pt, ws);
        hipLaunchKernelGGL(k_pauli_tiled_finish, dim3(1), dim3(kRedThreads), 0, s, ws, (int)nb,
                           nterms, coef_dev, ny_dev, out_dev);
        return hipGetLastError();
    }
    // split groups into chunks of <= 8 terms
    std::size_t nch = 0;
    for (int g = 0; g < ngroups; ++g) nch += (groups[g].count + kPauliChunk - 1) / kPauliChunk;
    if (nch == 0) {
        const double zero[2] = {0.0, 0.0};
        return hipMemcpyAsync(out_dev, zero, sizeof(zero), hipMemcpyHostToDevice, s);
    }
    PauliChunk *hc = new PauliChunk[nch];
    std::size_t c = 0;
    for (int g = 0; g < ngroups; ++g) {
        for (int f = 0; f < groups[g].count; f += kPauliChunk) {
            PauliChunk &ch = hc[c++];
            ch.x = groups[g].x;
            ch.hbit = ch.x ? 63 - __builtin_clzll(ch.x) : -1;
            ch.nt = groups[g].count - f < kPauliChunk ? groups[g].count - f : kPauliChunk;
            for (int t = 0; t < kPauliChunk; ++t)
                ch.term[t] = (t < ch.nt) ? groups[g].first + f + t : groups[g].first;
        }
    }
    const uint64_t work = (1ull << nq) / 2 + 1;
    uint64_t nb = (work + kRedThreads - 1) / kRedThreads;
    if (nb > kPauliBlocks) nb = kPauliBlocks;
    const size_t need = sizeof(double) * 2 * kPauliChunk * nb * nch + sizeof(PauliChunk) * nch;
    if (need > ws_bytes) {
        delete[] hc;
        return hipErrorInvalidValue;
    }
    double *partial = ws;
    PauliChunk *dch = (PauliChunk *)(ws + 2 * kPauliChunk * nb * nch);
    hipError_t e = hipMemcpyAsync(dch, hc, sizeof(PauliChunk) * nch, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // hc is freed below
    delete[] hc;
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)nb, (unsigned)nch);
    if (dtype == 0)
        hipLaunchKernelGGL(k_pauli<double>, grid, dim3(kRedThreads), 0, s, (const double2 *)psi,
                           nq, dch, z_dev, partial);
    else
        hipLaunchKernelGGL(k_pauli<float>, grid, dim3(kRedThreads), 0, s, (const float2 *)psi,
                           nq, dch, z_dev, partial);
    hipLaunchKernelGGL(k_pauli_finish, dim3(1), dim3(kRedThreads), 0, s, partial, (int)nch,
                       (int)nb, dch, coef_dev, ny_dev, out_dev);
    return hipGetLastError();
}

// --------------------------------------------------------------- sampling
// Blocks of 2^kSampleBits amplitudes: block sums and last nonzero index, an
// exclusive scan of the block sums, then one workgroup per shot resolves the
// index inside its block.
constexpr int kSampleBits = 12;

template <typename R>
__global__ __launch_bounds__(256) void k_block_sums(const typename V2r<R>::T *psi, int bbits,
                                                    double *bsum, int64_t *blast) {
    __shared__ double sh[16];
    __shared__ int64_t shl[4];
    const uint64_t b0 = (uint64_t)blockIdx.x << bbits;
    const int per = (1 << bbits) / 256 > 0 ? (1 << bbits) / 256 : 1;
    double acc = 0.0;
    int64_t last = -1;
    // lanes read consecutive amplitudes (coalesced); the order of the sum
    // need not match the in-block scan of k_sample, which settles a draw
    // that lands past its block's rounded end on the block's last nonzero
    for (int j = 0; j < per; ++j) {
        const uint32_t l = (uint32_t)j * 256u + threadIdx.x;
        if (l >= (1u << bbits)) break;
        const auto a = psi[b0 + l];
        const double p = (double)a.x * a.x + (double)a.y * a.y;
        acc += p;
        if (p > 0.0) last = (int64_t)(b0 + l);
    }
    acc = block_sum(acc, sh);
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t other = __shfl_down(last, o, 64);
        last = other > last ? other : last;
    }
    if ((threadIdx.x & 63) == 0) shl[threadIdx.x >> 6] = last;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t m = shl[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = shl[w] > m ? shl[w] : m;
        bsum[blockIdx.x] = acc;
        blast[blockIdx.x] = m;
    }
}

// Exclusive scan of nb block sums into prefix[0..nb] (prefix[nb] = total),
// and the largest nonzero index into *glast.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan(const double *bsum, const int64_t *blast,
                                               uint64_t nb, double *prefix, int64_t *glast) {
    __shared__ double sh[1024];
    __shared__ int64_t shl[1024];
    const uint64_t per = (nb + 1023) / 1024;
    const uint64_t lo = threadIdx.x * per;
    const uint64_t hi = lo + per < nb ? lo + per : nb;
    double s = 0.0;
    int64_t last = -1;
    for (uint64_t i = lo; i < hi; ++i) {
        s += bsum[i];
        last = blast[i] > last ? blast[i] : last;
    }
    sh[threadIdx.x] = s;
    shl[threadIdx.x] = last;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        int64_t m = -1;
        for (int t = 0; t < 1024; ++t) {
            const double v = sh[t];
            sh[t] = run;
            run += v;
            m = shl[t] > m ? shl[t] : m;
        }
        prefix[nb] = run;
        *glast = m;
    }
    __syncthreads();
    double run = sh[threadIdx.x];
    for (uint64_t i = lo; i < hi; ++i) {
        prefix[i] = run;
        run += bsum[i];
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_sample(const typename V2r<R>::T *psi, int bbits,
                                                uint64_t nb, const double *prefix,
                                                const int64_t *glast, const double *u,
                                                uint64_t *out) {
    __shared__ double sh[256];
    __shared__ uint64_t blk_s;
    __shared__ unsigned long long found;
    __shared__ long long lastnz;
    const double total = prefix[nb];
    const double r = u[blockIdx.x] * total;
    if (threadIdx.x == 0) {
        // first block whose end prefix exceeds r
        uint64_t lo = 0, hi = nb;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (prefix[mid + 1] > r) hi = mid;
            else lo = mid + 1;
        }
        blk_s = lo;
        found = ~0ull;
        lastnz = -1;
    }
    __syncthreads();
    const uint64_t blk = blk_s;
    if (blk >= nb) {
        if (threadIdx.x == 0) out[blockIdx.x] = (uint64_t)(*glast < 0 ? 0 : *glast);
        return;
    }
    const int bsize = 1 << bbits;
    const int per = bsize / 256 > 0 ? bsize / 256 : 1;
    const uint64_t b0 = blk << bbits;
    double seg = 0.0;
    for (int j = 0; j < per; ++j) {
        const int l = threadIdx.x * per + j;
        if (l >= bsize) break;
        const auto a = psi[b0 + l];
        seg += (double)a.x * a.x + (double)a.y * a.y;
    }
    sh[threadIdx.x] = seg;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int t = 0; t < 256; ++t) {
            const double v = sh[t];
            sh[t] = run;
            run += v;
        }
    }
    __syncthreads();
    double c = prefix[blk] + sh[threadIdx.x];
    for (int j = 0; j < per; ++j) {
        const int l = threadIdx.x * per + j;
        if (l >= bsize) break;
        const auto a = psi[b0 + l];
        const double p = (double)a.x * a.x + (double)a.y * a.y;
        c += p;
        if (p > 0.0) atomicMax(&lastnz, (long long)(b0 + l));
        if (c > r) {
            atomicMin(&found, (unsigned long long)(b0 + l));
            break;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t res = found;
        if (res == ~0ull) res = lastnz >= 0 ? (uint64_t)lastnz : (uint64_t)(*glast < 0 ? 0 : *glast);
        out[blockIdx.x] = res;
    }
}

size_t sample_workspace_bytes(int nq) {
    const int bb = nq < kSampleBits ? nq : kSampleBits;
    const uint64_t nb = 1ull << (nq - bb);
    return sizeof(double) * (2 * nb + 2) + sizeof(int64_t) * (nb + 2);
}

hipError_t sample(int dtype, const void *psi, int nq, int shots, const double *u_dev,
                  double *ws, uint64_t *out_dev, hipStream_t s) {
    const int bb = nq < kSampleBits ? nq : kSampleBits;
    const uint64_t nb = 1ull << (nq - bb);
    double *bsum = ws;
    double *prefix = ws + nb;
    int64_t *blast = (int64_t *)(prefix + nb + 2);
    int64_t *glast = blast + nb;
    if (dtype == 0)
        hipLaunchKernelGGL(k_block_sums<double>, dim3((unsigned)nb), dim3(256), 0, s,
                           (const double2 *)psi, bb, bsum, blast);
    else
        hipLaunchKernelGGL(k_block_sums<float>, dim3((unsigned)nb), dim3(256), 0, s,
                           (const float2 *)psi, bb, bsum, blast);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, bsum, blast, nb, prefix, glast);
    if (shots > 0) {
        if (dtype == 0)
            hipLaunchKernelGGL(k_sample<double>, dim3(shots), dim3(256), 0, s,
                               (const double2 *)psi, bb, nb, prefix, glast, u_dev, out_dev);
        else
            hipLaunchKernelGGL(k_sample<float>, dim3(shots), dim3(256), 0, s,
                               (const float2 *)psi, bb, nb, prefix, glast, u_dev, out_dev);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ state ops
template <typename R>
__global__ void k_fill_basis0(typename V2r<R>::T *psi, uint64_t dim) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        typename V2r<R>::T v;
        v.x = (i == 0) ? R(1) : R(0);
        v.y = R(0);
        psi[i] = v;
    }
}

template <typename R>
__global__ void k_zero(typename V2r<R>::T *psi, uint64_t from, uint64_t to) {
    for (uint64_t i = from + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < to;
         i += (uint64_t)gridDim.x * blockDim.x) {
        typename V2r<R>::T v;
        v.x = R(0);
        v.y = R(0);
        psi[i] = v;
    }
}

template <typename R>
__global__ void k_compact(const typename V2r<R>::T *src, typename V2r<R>::T *dst, uint64_t half,
                          int q, int value) {
    const uint64_t lowm = (1ull << q) - 1;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < half;
         j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = ((j & ~lowm) << 1) | (j & lowm) | ((uint64_t)value << q);
        dst[j] = src[i];
    }
}

template <typename R>
__global__ void k_collapse(typename V2r<R>::T *psi, uint64_t dim, int q, int outcome,
                           double scale) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        auto a = psi[i];
        if ((int)((i >> q) & 1) == outcome) {
            a.x = (R)((double)a.x * scale);
            a.y = (R)((double)a.y * scale);
        } else {
            a.x = R(0);
            a.y = R(0);
        }
        psi[i] = a;
    }
}

template <typename R>
__global__ void k_gather(const typename V2r<R>::T *psi, const uint64_t *idx, uint64_t count,
                         double *out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const auto a = psi[idx[i]];
        out[2 * i] = (double)a.x;
        out[2 * i + 1] = (double)a.y;
    }
}

template <typename RS, typename RD>
__global__ void k_convert(const typename V2r<RS>::T *src, typename V2r<RD>::T *dst,
                          uint64_t dim) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const auto a = src[i];
        typename V2r<RD>::T b;
        b.x = (RD)a.x;
        b.y = (RD)a.y;
        dst[i] = b;
    }
}

// Elementwise kernels stride over their range; the grid is capped at 2^20
// blocks of 256 so that grid x block stays far below 2^32 threads at 2^33
// amplitudes.
static dim3 g1(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    if (b > (1ull << 20)) b = 1ull << 20;
    return dim3((unsigned)(b ? b : 1));
}

hipError_t fill_basis0(int dtype, void *psi, uint64_t dim, hipStream_t s) {
    if (dtype == 0)
        hipLaunchKernelGGL(k_fill_basis0<double>, g1(dim), dim3(256), 0, s, (double2 *)psi, dim);
    else
        hipLaunchKernelGGL(k_fill_basis0<float>, g1(dim), dim3(256), 0, s, (float2 *)psi, dim);
    return hipGetLastError();
}

hipError_t zero_range(int dtype, void *psi, uint64_t from, uint64_t to, hipStream_t s) {
    if (to <= from) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL(k_zero<double>, g1(to - from), dim3(256), 0, s, (double2 *)psi, from,
                           to);
    else
        hipLaunchKernelGGL(k_zero<float>, g1(to - from), dim3(256), 0, s, (float2 *)psi, from,
                           to);
    return hipGetLastError();
}

hipError_t compact(int dtype, const void *src, void *dst, int nq, int q, int value,
                   hipStream_t s) {
    const uint64_t half = 1ull << (nq - 1);
    if (dtype == 0)
        hipLaunchKernelGGL(k_compact<double>, g1(half), dim3(256), 0, s, (const double2 *)src,
                           (double2 *)dst, half, q, value);
    else
        hipLaunchKernelGGL(k_compact<float>, g1(half), dim3(256), 0, s, (const float2 *)src,
                           (float2 *)dst, half, q, value);
    return hipGetLastError();
}

hipError_t collapse(int dtype, void *psi, int nq, int q, int outcome, double scale,
                    hipStream_t s) {
    const uint64_t dim = 1ull << nq;
    if (dtype == 0)
        hipLaunchKernelGGL(k_collapse<double>, g1(dim), dim3(256), 0, s, (double2 *)psi, dim, q,
                           outcome, scale);
    else
        hipLaunchKernelGGL(k_collapse<float>, g1(dim), dim3(256), 0, s, (float2 *)psi, dim, q,
                           outcome, scale);
    return hipGetLastError();
}

hipError_t gather(int dtype, const void *psi, const uint64_t *idx, uint64_t count,
                  double *out, hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL(k_gather<double>, g1(count), dim3(256), 0, s, (const double2 *)psi, idx,
                           count, out);
    else
        hipLaunchKernelGGL(k_gather<float>, g1(count), dim3(256), 0, s, (const float2 *)psi, idx,
                           count, out);
    return hipGetLastError();
}

hipError_t convert_state(int ds, const void *src, int dd, void *dst, uint64_t dim,
                         hipStream_t s) {
    if (ds == 0 && dd == 1)
        hipLaunchKernelGGL((k_convert<double, float>), g1(dim), dim3(256), 0, s,
                           (const double2 *)src, (float2 *)dst, dim);
    else if (ds == 1 && dd == 0)
        hipLaunchKernelGGL((k_convert<float, double>), g1(dim), dim3(256), 0, s,
                           (const float2 *)src, (double2 *)dst, dim);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace dev
}  // namespace qsv
