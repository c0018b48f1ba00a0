// Plain-data descriptors passed from the host runtime to the HIP kernels, and
// the launcher entry points (implemented in the .hip files).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace qsv {
namespace dev {

// Index expansion: a group id g becomes an amplitude index by inserting a 0
// bit at each of the npos sorted positions, then OR-ing `ones`.
struct IndexArgs {
    uint64_t ones = 0;
    int32_t npos = 0;
    uint8_t pos[64] = {};
};

// Dense k-qubit matrix for the per-gate kernels, k <= 3, passed by value.
struct DenseArgs {
    double mr[64];    // row-major 2^k x 2^k, real parts
    double mi[64];    // imaginary parts
    uint64_t off[8];  // amplitude offset of matrix index r
};

// Monomial matrix: row r takes val[r] * x[src[r]]; only rows in `touch`.
struct MonoArgs {
    double vr[32], vi[32];
    uint64_t off[32];     // offset of row r
    uint64_t srcoff[32];  // offset of the column feeding row r
    uint32_t touch;
};

// One operation inside an LDS-tile pass.  Local positions index the tile
// (bit i of the local index <-> i-th lowest tile position).
// TOP_DENSE_MFMA: dense k = 3..5 op on matrix cores; `mat` then points at
// the real embedding W = [[Re U, -Im U], [Im U, Re U]] (2^(k+1) x 2^(k+1),
// row-major, in the tile's real type).
enum TileOpKind : int32_t { TOP_DENSE = 0, TOP_MONO = 1, TOP_DIAG_GLOBAL = 2, TOP_DENSE_MFMA = 3 };
struct TileOp {
    int32_t kind;
    int32_t k;
    int32_t nfree;        // group bits: tile bits that are neither targets nor local controls
    uint32_t touch;       // MONO / DIAG: rows that change
    uint64_t ectrl;       // control bits outside the tile: the op runs only if all are 1
    uint64_t gctrl;       // DIAG_GLOBAL: control mask over the global index
    uint32_t gt[8];       // DIAG_GLOBAL: global target positions
    // Byte offsets in the XOR-swizzled LDS tile.  The swizzle is linear over
    // GF(2) in the local index, so the address of row r of group g is
    // sl[r] XOR (XOR of fz[b] over the set bits b of g).
    uint32_t fz[16];      // free bit b (free bits in ascending local position)
    uint32_t sl[32];      // row r: its target bits, plus the local controls
    uint32_t ss[32];      // MONO: the row feeding row r
    int64_t mat;          // offset (in complex entries of the tile dtype) into the pool
};

struct TileArgs {
    int32_t m;            // tile bits
    int32_t n_ops;
    int32_t nq;           // state qubits
    int32_t tile_pos_n;   // == m
    uint32_t tpos[40];    // tile positions, ascending (words: uniform indexed loads stay scalar)
    uint64_t n_tiles;
    int32_t rb;           // register bits per thread (threads = 2^(m - rb))
    int32_t mfma_k;       // LDS kernel: widest matrix-core op of the pass (0 = none)
    int32_t no_diag;      // register kernel: 1 if the program has no ROP_DIAG op (a
                          // leaner kernel instance without that case runs it)
    uint32_t img_bytes;   // register kernel: bytes of the pass's LDS image (multiple of 16)
    int32_t store_sync;   // register kernel: 1 = workgroup barrier between the ops and the
                          // stores (the stores go where other threads loaded)
    int64_t img_off;      // register kernel: byte offset of the LDS image in the pool
    uint64_t g_reg[8];    // register kernel, layout at load time: global index bit of
                          // register bit j, and of thread-id bit i
    uint64_t g_thr[16];
    uint64_t g_reg_f[8];  // register kernel, layout at store time (after the last remap)
    uint64_t g_thr_f[16];
    uint64_t dep_hi[64];  // LDS kernel: global offset of local index 256 * i (tile bits >= 8)
    uint32_t spos[40];    // LDS kernel, stores: position of tile bit i (== tpos[i] unless
                          // the pass relabels its qubits)
    uint64_t dep_hi_f[64];// LDS kernel, stores: dep_hi over spos
};

// One operation of the register-resident tile kernel.
//   G1/G2: complex 1- or 2-qubit matrix on register bits.
//   R1/R2: real 1- or 2-qubit matrix on register bits (a complex matrix that
//          is real up to diagonal phases on either side; the phases become
//          DIAG ops), half the arithmetic of G1/G2 per amplitude.
//   DIAG:  per-amplitude factor from a table in the pass's LDS image.
//   REMAP: layout change through the LDS half-tile buffer.
enum RegOpKind : int32_t { ROP_G1 = 0, ROP_G2 = 1, ROP_DIAG = 2, ROP_REMAP = 3, ROP_R1 = 5, ROP_R2 = 6 };
// Widest diagonal op of the register kernel (table bits; its table of 2^k
// factors lives in the pass's LDS image).
constexpr int kRegDiagMax = 8;
// LDS-image bytes of a register pass (tables and per-lane words): the
// lowering narrows the tables to stay within kRegImageSoft where it can; a
// larger image lowers occupancy; past kRegImageMax the pass runs on the
// LDS-tile kernel.
constexpr uint32_t kRegImageSoft = 20480;
constexpr uint32_t kRegImageMax = 65536;

// The LDS image of a register pass holds the DIAG tables (each aligned to its
// own size, in the state's complex type) and, for each REMAP, 32-bit words:
// the buffer write offsets of the 64 lanes' thread-id bits, then their read
// offsets.  The wave's part of the same offsets is uniform (wwave/rwave).
struct RegOp {
    int32_t kind;
    int32_t a;            // G1/R1: register bit; G2/R2: lower register bit (matrix bit 0);
                          // REMAP: register slot whose tile bit stays put;
                          // DIAG: number of table bits outside the tile
    int32_t b;            // G2/R2: higher register bit (matrix bit 1); DIAG: byte offset
                          // of a table of ones, read by tiles that fail `octrl`
    uint32_t creg;        // G/R: register bits that are controls (mask over register index)
    uint64_t octrl;       // controls outside the tile: the op runs on a tile only if its
                          // base index has all these bits
    uint64_t lane_ok;     // G/R: bit l set if lane l meets the controls on thread-id bits;
                          // DIAG: bit t set if lane bit t (thread-id bit t < 6) is a
                          // table bit, rd[t] then its place in the table byte offset
    uint32_t wave_ok;     // G/R: bit w set if wave w meets them
    uint32_t lane_off;    // REMAP: byte offset of the op's per-lane words in the image
    int64_t mat;          // DIAG: byte offset of the factor table in the image
    // The payload of the op's kind.  An op is read through the scalar cache
    // for every tile, so it keeps to few 64-byte lines: the two kinds share
    // storage, the fields a kind reads with the header come first, and the
    // size is a whole number of lines (448 bytes; programs start on 256).
    union {
        struct {
            // G/R: the matrix, row-major over (bit 0 <-> a, bit 1 <-> b),
            // inline so that one burst of scalar loads brings an op's fields
            // and its matrix: R1 4 and R2 16 reals, G1 4 and G2 16 complex
            // (re, im); in double for a complex128 state (md) and in float
            // for complex64 (mf)
            double md[32];
            float mf[32];
        };
        struct {
            uint32_t gt[8];       // DIAG: global positions of the table bits outside the tile
            uint32_t gtb[8];      //       and their byte weights in the table
            uint32_t wwave[8];    // DIAG: table byte offset of the wave's thread-id bits;
                                  // REMAP: write offset of the wave's thread-id bits
            uint32_t rwave[8];    // REMAP: read offset of the wave's thread-id bits
            uint32_t wr[32];      // DIAG: table byte offset of register index i;
                                  // REMAP: buffer byte offset of register i in the old layout
            uint32_t rd[32];      // REMAP: buffer byte offset of register i in the new layout;
                                  // DIAG: see lane_ok
        };
    };
    uint32_t pad_[4];
};
static_assert(sizeof(RegOp) % 64 == 0, "register ops start on scalar cache lines");

// A run of work items of one batched register-tile launch that belong to one
// circuit's pass: item - first = tile index; the pass's TileArgs (tile
// positions, layouts, image) at tas[ta], its program at rops[op_begin].
struct RegSeg {
    uint64_t first;
    uint64_t state_off;
    int32_t ta;
    int32_t op_begin;
};

// ------------------------------------------------------------------ gates
// dtype: 0 = complex128, 1 = complex64.  Sizes in amplitudes.
hipError_t launch_dense(int dtype, void *psi, int k, uint64_t ngroups, const IndexArgs &ia,
                        const DenseArgs &a, hipStream_t s);
hipError_t launch_mono(int dtype, void *psi, int k, uint64_t ngroups, const IndexArgs &ia,
                       const MonoArgs &a, hipStream_t s);
hipError_t launch_tile_pass(int dtype, void *psi, const TileArgs &ta, const TileOp *ops,
                            const void *pool, unsigned int *counter, hipStream_t s);
// Register-resident tile pass: ta.rb register bits in {3, 4, 5} and
// ta.m - ta.rb thread bits in {8, 9}.  `counter` is a device word that must
// hold 0 when the pass starts; the persistent workgroups take tiles from it.
// Batched register-tile launch (12-bit tiles, 16 amplitudes per thread):
// items work items over the segments, a fixed stride per workgroup; img_max:
// the largest image of the segments' passes.
hipError_t launch_tile_reg_batch(int dtype, bool dg, void *states, const RegSeg *segs, int nseg,
                                 uint64_t items, const TileArgs *tas, const RegOp *rops,
                                 const void *pool, uint32_t img_max, hipStream_t s);
hipError_t launch_tile_reg(int dtype, void *psi, const TileArgs &ta, const RegOp *rops,
                           const void *pool, unsigned int *counter, hipStream_t s);
int tile_pass_max_bits(int dtype);
int tile_reg_bits(int dtype);     // default register bits per thread

// Streaming copy of `bytes` (a multiple of 16) from src to dst (the
// bandwidth probe).
hipError_t copy_probe(const void *src, void *dst, uint64_t bytes, hipStream_t s);

// ------------------------------------------------------------ state ops
hipError_t fill_basis0(int dtype, void *psi, uint64_t dim, hipStream_t s);
hipError_t zero_range(int dtype, void *psi, uint64_t from, uint64_t to, hipStream_t s);
hipError_t compact(int dtype, const void *src, void *dst, int nq, int q, int value,
                   hipStream_t s);
hipError_t collapse(int dtype, void *psi, int nq, int q, int outcome, double scale,
                    hipStream_t s);
hipError_t gather(int dtype, const void *psi, const uint64_t *idx, uint64_t count,
                  double *out, hipStream_t s);
hipError_t convert_state(int dtype_src, const void *src, int dtype_dst, void *dst,
                         uint64_t dim, hipStream_t s);

// -------------------------------------------------------------- reductions
// Workspace needs: see reduce_workspace_bytes().
size_t reduce_workspace_bytes(int nq);
// Sum of |psi_i|^2 over the indices matching (ia): out_dev[0].
hipError_t prob_masked(int dtype, const void *psi, uint64_t ngroups, const IndexArgs &ia,
                       double *ws, double *out_dev, hipStream_t s);
// The same with the partial sums in a static device array of the library
// (no allocation); hipErrorInvalidValue if they would not fit.
hipError_t prob_masked_noalloc(int dtype, const void *psi, uint64_t ngroups, const IndexArgs &ia,
                               double *out_dev, hipStream_t s);
int prob_noalloc_partials(uint64_t ngroups);   // partial sums a call needs
int prob_noalloc_capacity();                   // partial sums the array holds
// p0 (bit q = 0) and p1 (bit q = 1): out_dev[0..1].
hipError_t prob_split(int dtype, const void *psi, int nq, int q, double *ws, double *out_dev,
                      hipStream_t s);
hipError_t probs(int dtype, const void *psi, uint64_t dim, double *out_dev, hipStream_t s);
// Reduced density matrix of the k <= 2 qubits at bit positions pos[0..k-1]:
// out_dev[2 * (a * 2^k + b) + {0, 1}] = re / im of sum over the other bits of
// psi[i_a] conj(psi[i_b]), where bit j of a is the bit at pos[j] of i_a.
// Accumulated in double; ws holds reduced_dm_workspace_bytes().
hipError_t reduced_dm(int dtype, const void *psi, int nq, int k, const int *pos, double *ws,
                      double *out_dev, hipStream_t s);
size_t reduced_dm_workspace_bytes();

// Pauli sum.  Terms are grouped by x mask on the host; `grp_*` describe the
// groups.  out_dev[0..1] = sum_t coeff_t <P_t> (re, im).
struct PauliGroup {
    uint64_t x;
    int32_t first;        // first term index of the group
    int32_t count;        // terms in the group
};
hipError_t pauli_expectation(int dtype, const void *psi, int nq, int ngroups,
                             const PauliGroup *groups_host, const uint64_t *z_dev,
                             const double *coef_dev, const int32_t *ny_dev, int nterms,
                             double *ws, size_t ws_bytes, double *out_dev, hipStream_t s,
                             const uint64_t *z_host = nullptr);   // z masks on the host (same
                                                                  // order): enables the one-read
                                                                  // tiled path
size_t pauli_workspace_bytes(int nq, int ngroups, int nterms);

// ---------------------------------------------------------------- adjoint
// phi = H psi for a Pauli sum over bit positions (device arrays).
hipError_t ham_apply(int dtype, const void *psi, void *phi, uint64_t dim, int nterms,
                     const uint64_t *x, const uint64_t *z, const double *c, const int32_t *ny,
                     hipStream_t s);
// out_dev[0] = Re<a|b>; ws holds adjoint_blocks(dim) doubles.
hipError_t dot_re(int dtype, const void *a, const void *b, uint64_t dim, double *ws,
                  double *out_dev, hipStream_t s);
int adjoint_blocks(uint64_t npairs);
// Reverse step for exp(-i theta P/2), P = X/Y/Z (axis 1/2/3), on the pairs
// given by ia (target bit cleared, controls set) and partner offset toff;
// c = cos(theta/2), sn = sin(theta/2).  Runs nb workgroups and writes
// partial[0..nb) (one sum per workgroup, zero for those without pairs), so
// that rows of rotations with and without controls have the same width.
hipError_t adjoint_rotation(int dtype, void *psi, void *phi, uint64_t npairs,
                            const IndexArgs &ia, uint64_t toff, int axis, double c, double sn,
                            double *partial, int nb, hipStream_t s);
// grad[p] = sum over rotations g with param[g] = p of sum_b partial[g * nb + b]
// (the rows are summed in place; their first entries are overwritten).
hipError_t grad_finish(double *partial, int ng, int nb, const int32_t *param, double *grad,
                       int nparams, hipStream_t s);

// ---------------------------------------------------------------- batched
struct BatchCircuit {
    int32_t n;            // qubits
    int32_t pass_begin;   // first BatchPass
    int32_t pass_count;
    int32_t term_begin;   // first BatchTerm
    int32_t term_count;
    int32_t out_index;
    int32_t pad[2];
};
struct BatchPass {
    int32_t m;            // tile bits
    int32_t op_begin;     // first TileOp
    int32_t op_count;
    int32_t pad;
    uint32_t tpos[16];    // tile positions, ascending
};
struct BatchTerm {
    uint64_t x, z;
    double c;
    int32_t ny;
    int32_t pad;
};
// A run of consecutive work items of one launch that belong to one circuit:
// a pass's tiles (item - first = tile index) or a state's Pauli chunks
// (item - first = chunk index).  Segments of a launch are ordered by first.
struct BatchSeg {
    uint64_t first;
    uint64_t state_off;       // amplitude offset of the circuit's state in `states`
    int32_t pass;             // pass launches: the BatchPass
    int32_t circuit;          // the BatchCircuit
    int32_t init;             // 1: the circuit's first pass (tiles start from |0...0>)
    int32_t pad;
};
struct BatchLaunch {
    const BatchCircuit *circuits;
    const int32_t *order;     // processing order (longest first)
    int32_t count;
    const BatchPass *passes;
    const TileOp *ops;
    const void *pool;         // matrices in the batch dtype
    const BatchTerm *terms;
    void *scratch;            // grid slots of slot_amps amplitudes
    uint64_t slot_amps;
    int32_t mb;               // LDS-resident limit and tile bits
    unsigned int *counter;
    double *out;
    unsigned int grid;
    int32_t mfma_k;           // widest matrix-core op (0 = none), at most 5
    // Pass-major circuits (more qubits than the LDS holds), each with its
    // state in its own region of `states`: launch i < n_pass_launches runs
    // pass i of every such circuit that has one, over all its tiles; launch
    // n_pass_launches forms the Pauli sums in chunks; a last kernel adds each
    // circuit's chunk sums in order.  Launch i takes segments
    // [seg_begin[i], seg_begin[i + 1]) of `segs` and items[i] work items
    // (host arrays).  count above then counts only the circuits of k_batch.
    int32_t pass_major;       // 0: no pass-major circuits
    int32_t n_pass_launches;  // LDS-tile pass launches
    const BatchSeg *segs;
    const int32_t *seg_begin; // host, n_pass_launches + 2 entries
    const uint64_t *items;    // host, n_pass_launches + 1 entries
    void *states;
    double *partial;          // one sum per Pauli work item
    int32_t chunk_log;        // Pauli chunk: 2^chunk_log amplitudes (pairs for X strings)
    unsigned int grid_big;
    // Pass-major circuits of at least 13 qubits run on the register-tile
    // kernel (12-bit tiles, the planning and lowering of the single-state
    // path): their states (reg_amps amplitudes from amplitude reg_state_off
    // of `states`, each starting at reg_starts[i]) are set to |0...0> first,
    // then launch i < n_reg_launches runs segments [reg_seg_begin[i],
    // reg_seg_begin[i + 1]) of reg_segs over reg_items[i] tiles, with the
    // table-op instance where reg_dg[i].
    int32_t n_reg_launches;
    const RegSeg *reg_segs;
    const int32_t *reg_seg_begin; // host
    const uint64_t *reg_items;    // host
    const int32_t *reg_dg;        // host
    const TileArgs *tas;
    const RegOp *rops;
    const void *reg_pool;         // LDS images
    uint32_t reg_img_max;
    uint64_t reg_state_off, reg_amps;
    const uint64_t *reg_starts;
    int32_t n_reg_states;
};
hipError_t batch_launch(int dtype, const BatchLaunch &L, hipStream_t s);
int batch_occupancy(int dtype, int mb, int mfma_k);   // resident workgroups per CU
int batch_pass_occupancy(int dtype, int mb, int mfma_k);

// Sampling: out_dev[shots] indices.
size_t sample_workspace_bytes(int nq);
hipError_t sample(int dtype, const void *psi, int nq, int shots, const double *u_dev,
                  double *ws, uint64_t *out_dev, hipStream_t s);

}  // namespace dev
}  // namespace qsv
