/*
 * qsv.h -- C ABI of libqsv, a state-vector simulator core for AMD Instinct
 * MI355X (gfx950).
 *
 * The operations follow the problem statement of the ProjectQ paper
 * (Steiger, Haener, Troyer, arXiv:1612.08091):
 *   - qubits are allocated and deallocated at any time (Sec. 4.1.1); a qubit in
 *     superposition may not be deallocated (Sec. 4.1.1, the simulator raises);
 *   - gates are applied to qubits, optionally conditioned on control qubits
 *     being |1> (Sec. 4 "Gate | qubits" syntax; Sec. 4.1.3 Control);
 *   - the simulator evaluates gates lazily and executes them on flush
 *     (Sec. 4.1.3 eng.flush(); Sec. 4.3.2 "lazy evaluation of gates");
 *   - measurement in the computational basis, with results read back after a
 *     flush (Sec. 4, minimal example; App. A.1);
 *   - probabilities, Pauli-sum expectation values and sampling of the state,
 *     an adjoint gradient and a batched form are extensions of the same state
 *     vector (they do not appear in the paper).
 *
 * Conventions
 *   - A state of n qubits is 2^n complex amplitudes, interleaved (re, im), in
 *     double (QSV_C128) or float (QSV_C64).  The live qubit at bit position p
 *     is the p-th live qubit in allocation order; new qubits take the next
 *     highest positions; deallocating a qubit removes its bit and shifts the
 *     higher ones down.
 *   - Qubit ids are small non-negative integers handed out by qsv_allocate
 *     (the lowest unused id, so ids are < n_max <= 64).
 *   - A k-qubit gate matrix is 2^k x 2^k complex128, row-major, interleaved;
 *     bit j of its row/column index belongs to targets[j].
 *   - Every call returns a qsv_status.  On failure the handle keeps its
 *     previous state and qsv_last_error() describes the failure until the next
 *     call on that handle.
 *   - A handle is not thread-safe; distinct handles are independent.  Device
 *     work runs asynchronously on the handle's HIP stream; faults from it are
 *     reported as QSV_EDEVICE by the next call that synchronises.
 *   - Ownership: callers own every array they pass; the library copies what it
 *     keeps.  The library owns its device buffers, except a borrowed state
 *     buffer (qsv_options.state), which the caller must keep alive until
 *     qsv_destroy.
 */
#ifndef QSV_H
#define QSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum qsv_status {
    QSV_OK = 0,
    QSV_EINVAL = 1,         /* bad argument: id, size, duplicate qubit, non-finite entry */
    QSV_ENOMEM = 2,         /* state would exceed the capacity or device memory */
    QSV_EDEVICE = 3,        /* a HIP call or kernel failed */
    QSV_ENOTCLASSICAL = 4,  /* deallocation of a qubit in superposition */
    QSV_ESTATE = 5,         /* NULL or destroyed handle, or a call out of order */
    QSV_EUNSUPPORTED = 6    /* valid request that this build does not implement */
} qsv_status;

typedef enum qsv_dtype { QSV_C128 = 0, QSV_C64 = 1 } qsv_dtype;

/* Execution modes of qsv_flush. */
typedef enum qsv_mode {
    QSV_MODE_PERGATE = 0,   /* one kernel per gate, no fusion */
    QSV_MODE_FUSED = 1,     /* gates fused into <= k_max-qubit unitaries, one kernel each */
    QSV_MODE_TILED = 2      /* fused gates grouped into LDS-tile passes over HBM */
} qsv_mode;

typedef struct qsv_options {
    int32_t n_max;          /* capacity in qubits, 1..36 */
    int32_t dtype;          /* qsv_dtype */
    int32_t mode;           /* qsv_mode */
    int32_t k_max;          /* fusion width 1..5 (modes FUSED and TILED) */
    int32_t tile_bits;      /* qubits per LDS tile in mode TILED, 0 = default */
    int32_t queue_limit;    /* flush automatically after this many queued gates, 0 = 4096 */
    void *stream;           /* hipStream_t used for all device work; NULL = null stream */
    void *state;            /* optional borrowed device buffer for the state */
    uint64_t state_bytes;   /* its size in bytes (>= 2^n_max amplitudes) */
    int32_t timing;         /* 1: bracket every kernel with HIP events (qsv_get_kernel_times) */
    int32_t reg_bits;       /* amplitudes per thread = 2^reg_bits in the register-resident
                               tile kernel (3..5; tile_bits - reg_bits thread bits must be
                               8 or 9), 0 = default */
    int32_t relabel;        /* mode TILED, 1 (default): a pass may move its qubits to other
                               bit positions within its tile, so that the positions every
                               tile holds carry qubits in use and tiles span few 2 MiB
                               pages; every flush ends with each qubit back at its own
                               position.  0: positions never move */
    uint64_t mem_limit;     /* bytes the state buffer may take; ENOMEM, decided before any
                               allocation, when it needs more.  0 (default): the device's
                               free memory (hipMemGetInfo) at the time of the allocation */
} qsv_options;

/* Kernel classes reported by qsv_get_kernel_times. */
typedef enum qsv_kernel_class {
    QSV_K_TILE = 0,         /* LDS-tile pass (one HBM read + write of the state) */
    QSV_K_DENSE = 1,        /* per-gate dense update */
    QSV_K_MONO = 2,         /* per-gate monomial (permutation / diagonal) update */
    QSV_K_REDUCE = 3,       /* reductions, collapse, sampling */
    QSV_K_COUNT = 4
} qsv_kernel_class;

typedef struct qsv_sim qsv_sim;

/* Statistics of the work enqueued since the last qsv_reset_stats. */
typedef struct qsv_stats {
    uint64_t gates;         /* original gates executed */
    uint64_t fused_ops;     /* operations after fusion */
    uint64_t passes;        /* HBM passes over the state (kernel launches on it) */
    uint64_t kernels;       /* all kernels launched */
    double alg_bytes;       /* algorithmic HBM bytes of those launches */
    double alg_flops;       /* algorithmic floating-point operations */
    double amp_gate_updates;/* sum over original gates of 2^n */
} qsv_stats;

/* Fill *opt with defaults: n_max 30, C128, mode TILED, k_max 2, tile_bits 0,
 * relabel 1. */
qsv_status qsv_options_default(qsv_options *opt);

/* Create a simulator holding 0 qubits (state |>).  No device memory is
 * touched until the first call that needs the state on the device.
 * EINVAL on a bad option; ENOMEM if a borrowed buffer is too small. */
qsv_status qsv_create(const qsv_options *opt, qsv_sim **out);

/* Destroy a handle and free what the library allocated.  NULL is accepted. */
qsv_status qsv_destroy(qsv_sim *sim);

/* Allocate `count` qubits in |0> (Sec. 4.1.1, allocate_qureg).  Their ids are
 * written to ids_out[count] (may be NULL).  ENOMEM if n + count > n_max. */
qsv_status qsv_allocate(qsv_sim *sim, int32_t count, int32_t *ids_out);

/* Deallocate qubit `id` (Sec. 4.1.1).  Flushes, then computes p0 and p1 of the
 * qubit; if p1 <= tau the qubit is |0>, if p0 <= tau it is |1>, with
 * tau = 1e-12 (C128) or 1e-6 (C64); the state is then compacted.  Otherwise
 * ENOTCLASSICAL and nothing changes. */
qsv_status qsv_deallocate(qsv_sim *sim, int32_t id);

/* Number of live qubits, and their ids in bit-position order (ids may be NULL;
 * it must hold n entries). */
qsv_status qsv_qubits(const qsv_sim *sim, int32_t *n, int32_t *ids);

/* Queue gate U (2^k x 2^k complex128, row-major, interleaved) on targets[k],
 * conditioned on controls[c] all being |1> (Sec. 4.1.3 Control).  The matrix
 * is copied.  EINVAL for k outside 1..5, unknown or repeated qubits, or
 * non-finite entries.  Nothing runs until a flush (Sec. 4.3.2 lazy evaluation);
 * the queue flushes itself when it reaches queue_limit gates. */
qsv_status qsv_apply(qsv_sim *sim, const double *U, int32_t k, const int32_t *targets,
                     int32_t c, const int32_t *controls);

/* Queue the diagonal gate diag(d[0], ..., d[2^k - 1]) on targets[k] under
 * controls[c] (Sec. 4: Gate | qubits, with a Control block): d holds 2^k
 * interleaved complex128 entries, bit j of the row index <-> targets[j].
 * The same as qsv_apply with the diagonal matrix; diagonal gates take the
 * kernels' diagonal paths either way.  EINVAL as qsv_apply, or d NULL. */
qsv_status qsv_apply_diag(qsv_sim *sim, const double *d, int32_t k, const int32_t *targets,
                          int32_t c, const int32_t *controls);

/* Emulated math gate (Sec. 4.3.3: a BasicMathGate such as AddConstant applied
 * as the classical function it computes instead of its gate decomposition).
 * The register is qubits[0..w-1] (qubit ids, qubits[0] the least significant
 * bit of the register value x); table[x] (2^w entries, host memory, copied)
 * is the new value, and must be a permutation of 0..2^w-1 so that the map is
 * unitary.  For every basis state whose controls[0..c-1] are all |1>, its
 * amplitude moves to the basis state holding table[x] in the register and
 * the same values elsewhere; the other amplitudes stay.  Flushes the queue,
 * then runs at once (a gather into a second state-sized device buffer that
 * the handle keeps, then a pointer swap, or a copy back into a borrowed
 * state).  EINVAL: w outside 1..26, unknown or repeated qubits, w + c above
 * the live qubits, NULL table, or a table that is not a permutation (checked
 * before anything runs); ENOMEM if the second buffer cannot be allocated. */
qsv_status qsv_apply_math(qsv_sim *sim, int32_t w, const int32_t *qubits, const uint32_t *table,
                          int32_t c, const int32_t *controls);

/* ---------------------------------------------------------------------- */
/* Density matrices (noise: Sec. 4.3.2 names stochastic noise models and a  */
/* density-matrix simulator as future work).  A handle with 2n live qubits  */
/* holds vec(rho) of an n-qubit density matrix: rho[r][c] at index          */
/* r + 2^n c, so bit positions 0..n-1 index the row and n..2n-1 the column; */
/* a fresh handle's |0..0> is rho = |0..0><0..0|.  System qubit j is bit    */
/* position j (row) and j + n (column); the calls below take system qubit   */
/* indices 0..n-1, not ids.  Gates and channels queue like qsv_apply and    */
/* run through the same fusion and tile passes (on 2n qubits).              */
/* ---------------------------------------------------------------------- */

/* Queue rho <- G rho G^dagger for G = U on targets[k] (k <= 2) controlled by
 * controls[c]: U on the row bits, conj(U) on the column bits.  EINVAL for an
 * odd number of live qubits, indices outside 0..n-1 or repeated, k outside
 * 1..2, c + k > n, or non-finite entries. */
qsv_status qsv_dm_apply(qsv_sim *sim, const double *U, int32_t k, const int32_t *targets,
                        int32_t c, const int32_t *controls);

/* Queue the channel rho <- sum_j K_j rho K_j^dagger on targets[k] (k <= 2):
 * kraus holds nk matrices of 2^k x 2^k (row-major, interleaved complex128).
 * The superoperator M[r' + 2^k c'][r + 2^k c] = sum_j K_j[r'][r]
 * conj(K_j[c'][c]) is formed on the host in complex128 and queued as one op
 * on the k row bits and the k column bits.  The
 * channel is taken as given (trace preservation is the caller's).  EINVAL as
 * qsv_dm_apply, or nk < 1, or non-finite entries. */
qsv_status qsv_dm_apply_kraus(qsv_sim *sim, int32_t nk, const double *kraus, int32_t k,
                              const int32_t *targets);

/* out[i] = Re rho[i][i] for i < 2^n (host memory): the probabilities of a
 * measurement of all qubits.  Flushes; synchronises. */
qsv_status qsv_dm_probabilities(qsv_sim *sim, double *out);

/* *out = sum_t coeff[t] Re Tr(rho P_t); masks over system qubits 0..n-1 as in
 * qsv_get_expectation_value (X only in xmask, Z only in zmask, Y in both).
 * Flushes; synchronises. */
qsv_status qsv_dm_expectation(qsv_sim *sim, int32_t nterms, const uint64_t *xmask,
                              const uint64_t *zmask, const double *coeff, double *out);

/* Execute every queued gate (Sec. 4.1.3 eng.flush()): plan fusion and passes,
 * enqueue the kernels on the stream.  Asynchronous.  The state is allocated
 * on first use: ENOMEM if it would not fit (mem_limit, else the device's free
 * memory, checked before allocating), with the queue and the register left as
 * they were (the handle can still be destroyed).  A failure after some of the
 * flush's kernels were enqueued drops the queue (its gates would otherwise
 * run twice) and leaves the state invalid: every call that needs it returns
 * EDEVICE until qsv_reset or qsv_set_state.  For tests of this path the
 * environment variable QSV_INJECT_LAUNCH_FAILURE=k, read by qsv_create, makes
 * the handle's launch number k (counted from 0) fail without launching. */
qsv_status qsv_flush(qsv_sim *sim);

/* Wait for the stream; EDEVICE if any enqueued work failed. */
qsv_status qsv_synchronize(qsv_sim *sim);

/* Sum of |psi_i|^2 over the indices where qubit qubits[j] has value bits[j]
 * for all j < m (m = 0: the squared norm).  Flushes; synchronises. */
qsv_status qsv_get_probability(qsv_sim *sim, int32_t m, const int32_t *qubits,
                               const int8_t *bits, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sum of
 * qsv_get_probability, computed by the same kernels on a caller-owned device
 * state of 2^n amplitudes (dtype QSV_C128 or QSV_C64, interleaved) over the
 * indices whose bit positions[j] equals bits[j] for all j < m (positions are
 * bit positions, not qubit ids; m = 0: the squared norm).  The double result
 * goes to the device address out_dev; the work is enqueued on `stream` (a
 * hipStream_t, NULL = null stream) and nothing synchronises.  No device
 * memory is allocated and no HIP allocation routine is called: the partial
 * sums (at most 1024 doubles, 8 KiB) live in a static device array of the
 * library, one per GPU, held until the process ends; every call writes the
 * slots it reads.  Calls that overlap on one GPU race on that array.
 * EINVAL: NULL pointer, bad dtype, n outside 0..36, m outside 0..n, a
 * position outside 0..n-1 or repeated, or partial sums beyond the array;
 * EDEVICE: a HIP call failed (qsv_last_error(NULL) says which). */
qsv_status qsv_get_probability_noalloc(const void *state, int32_t dtype, int32_t n, int32_t m,
                                       const int32_t *positions, const int8_t *bits,
                                       double *out_dev, void *stream);

/* All 2^n probabilities |psi_i|^2 as doubles into out (host memory if
 * out_is_device == 0, else a device pointer).  Flushes; synchronises. */
qsv_status qsv_get_probabilities(qsv_sim *sim, double *out, int32_t out_is_device);

/* <psi|H|psi> for H = sum_t coeff[t] P_t; P_t has X on the qubit ids set only
 * in xmask[t], Z on those only in zmask[t], Y on those in both (bit q of a mask
 * is qubit id q).  Accumulated in double.  *out = the real part; EINVAL if
 * an id is not live.  Flushes; synchronises. */
qsv_status qsv_get_expectation(qsv_sim *sim, int32_t nterms, const uint64_t *xmask,
                               const uint64_t *zmask, const double *coeff, double *out);

/* As qsv_get_expectation, with the imaginary part of sum_t coeff[t] <P_t> in
 * *im_out.  A Pauli sum with real coefficients is Hermitian, so the
 * imaginary part is zero up to rounding; it is returned so that callers (and
 * the parity tests) can check that.  Flushes; synchronises. */
qsv_status qsv_get_expectation_complex(qsv_sim *sim, int32_t nterms, const uint64_t *xmask,
                                       const uint64_t *zmask, const double *coeff, double *re_out,
                                       double *im_out);

/* Measure qubits[m] one after the other in list order (App. A.1), qubit j with
 * the caller's uniform u[j] in [0,1): outcome 0 iff u*(p0+p1) < p0; the other
 * branch is zeroed and the kept one scaled by 1/sqrt(p_outcome).  Outcomes go
 * to bits_out[m].  Flushes; synchronises. */
qsv_status qsv_measure(qsv_sim *sim, int32_t m, const int32_t *qubits, const double *u,
                       int8_t *bits_out);

/* One step of a stochastic noise trajectory (Sec. 4.3.2 names stochastic
 * noise models as future work): the channel with Kraus operators K_j
 * (kraus: nk matrices of 2^k x 2^k, row-major, interleaved complex128) on
 * targets[k], k <= 2, is replaced by one of its branches.  Branch j has
 * probability p_j = ||K_j psi||^2 = Tr(K_j rho_T K_j^dagger), rho_T the
 * reduced density matrix of the targets (one reduction over the state,
 * accumulated in double); the branch taken is the smallest j whose running
 * sum of p exceeds u * sum_j p_j (u in [0,1), the caller's uniform), and
 * K_j / sqrt(p_j) is queued as a gate, so the state keeps unit norm.
 * *chosen = j; probs[nk] (may be NULL) receives the p_j.  Averaged over u,
 * |psi><psi| follows the channel sum_j K_j rho K_j^dagger.  EINVAL for k
 * outside 1..2, unknown or repeated ids, u outside [0,1), non-finite
 * entries, or a channel that leaves no probability.  Flushes; synchronises. */
qsv_status qsv_apply_kraus_sampled(qsv_sim *sim, int32_t nk, const double *kraus, int32_t k,
                                   const int32_t *targets, double u, int32_t *chosen,
                                   double *probs);

/* Draw `shots` samples without collapse.  Shot s returns the smallest index i
 * with C_i > u[s] * T, C the running sum of |psi|^2 in double and T its total,
 * or the largest i with |psi_i|^2 > 0 if none.  out[s] has bit p = value of the
 * qubit at bit position p.  Flushes; synchronises. */
qsv_status qsv_sample(qsv_sim *sim, int32_t shots, const double *u, uint64_t *out);

/* Copy the 2^n amplitudes (the handle's dtype, interleaved) to / from a host
 * buffer (is_device == 0) or a device buffer.  get flushes first; set drops
 * any queued gates.  Both synchronise. */
qsv_status qsv_get_state(qsv_sim *sim, void *dst, int32_t dst_is_device);
qsv_status qsv_set_state(qsv_sim *sim, const void *src, int32_t src_is_device);

/* Gather count amplitudes psi[indices[i]] as complex128 (re, im) pairs into
 * the host array out[2*count] (used to check sampled amplitudes of large
 * states).  EINVAL for an index >= 2^n.  Flushes; synchronises. */
qsv_status qsv_get_amplitudes(qsv_sim *sim, int64_t count, const uint64_t *indices,
                              double *out);

/* Device pointer of the state and the handle's stream (for callers that
 * wrap the buffer, e.g. as a torch tensor).  Flushes. */
qsv_status qsv_state_pointer(qsv_sim *sim, void **ptr, void **stream);

/* Reset the state to |0...0> on the live qubits and drop queued gates. */
qsv_status qsv_reset(qsv_sim *sim);

/* With qsv_options.timing = 1: total device time (ms, from HIP events
 * recorded on the handle's stream around each launch), number of launches
 * and algorithmic HBM bytes of the kernels of class `kclass` since the last
 * qsv_reset_stats.  Synchronises. */
qsv_status qsv_get_kernel_times(qsv_sim *sim, int32_t kclass, double *ms, uint64_t *launches,
                                double *alg_bytes);

qsv_status qsv_get_stats(const qsv_sim *sim, qsv_stats *out);
qsv_status qsv_reset_stats(qsv_sim *sim);

/* Run the fusion and pass planners of the handle's mode on the queued gates
 * without executing them (the queue is kept).  Host only, no device call.
 * Writes the number of operations and passes; if max_ops > 0, also for
 * operation i < max_ops: its target count ks[i], its target bit positions
 * targets[5*i + j] (bit j of its matrix index), its control positions as a
 * mask ctrls[i], and its matrix over the targets in mats[i*2048 ...]
 * (2^k x 2^k complex128, row-major, interleaved).  Operations come out in
 * execution order; applying them one after the other equals applying the
 * queued gates. */
qsv_status qsv_plan(qsv_sim *sim, int32_t *n_ops, int32_t *n_passes, int32_t max_ops,
                    int32_t *ks, int32_t *targets, uint64_t *ctrls, double *mats);

/* Host-side check of the register-tile programs (the lowering behind the
 * bulk execution of cached gates, Sec. 4.3.2), for tests: plans the queued
 * gates as qsv_flush does in mode TILED, lowers every pass to the
 * instruction list of the register-resident tile kernel, and runs those
 * lists on the host over state[2 * 2^n] (complex128, interleaved, updated in
 * place) thread by thread, with the kernel's layouts, LDS byte offsets and
 * table lookups, every address bounds-checked.  state NULL: lower only (for
 * the counts).  No device call; the queue is kept.  info[10] (may be NULL)
 * receives: passes, register passes, real-split ops, table (diagonal) ops,
 * layout changes, largest LDS image in bytes, instructions, diagonal ops
 * merged into another, layout changes within each wave (no barrier), passes
 * that move qubits to other positions (option relabel).  The state comes
 * out with every qubit at its own position.  EINVAL: not in mode TILED, or an address check
 * failed (qsv_last_error names it); EUNSUPPORTED: a pass needs the LDS-tile
 * kernel (an op wider than 2 qubits, or too many tables). */
qsv_status qsv_check_tile_programs(qsv_sim *sim, double *state, int32_t *info);

/* ----------------------------------------------------------------------- */
/* Circuits with parameters, Pauli sums: flat arrays used by the adjoint      */
/* gradient and by the batched form.                                          */
/* ----------------------------------------------------------------------- */
typedef enum qsv_op {
    QSV_OP_MATRIX = 0,      /* fixed matrix from `matrices` */
    QSV_OP_RX = 1,          /* exp(-i theta X / 2), theta = params[param[g]] */
    QSV_OP_RY = 2,
    QSV_OP_RZ = 3
} qsv_op;

typedef struct qsv_circuit {
    int32_t n_qubits;
    int32_t n_gates;
    const int32_t *op;        /* [n_gates] qsv_op */
    const int32_t *k;         /* [n_gates] number of targets (1 for rotations) */
    const int32_t *c;         /* [n_gates] number of controls */
    const int32_t *qubits;    /* [n_gates * 8]: targets then controls, qubit = bit position */
    const int64_t *mat_off;   /* [n_gates] offset (in complex entries) into matrices, QSV_OP_MATRIX */
    const double *matrices;   /* complex128 interleaved */
    const int32_t *param;     /* [n_gates] parameter index for rotations, -1 otherwise */
    int32_t n_params;
    const double *params;     /* [n_params] angles */
} qsv_circuit;

typedef struct qsv_pauli_sum {
    int32_t n_terms;
    const uint64_t *xmask;    /* bit p = bit position p */
    const uint64_t *zmask;
    const double *coeff;
} qsv_pauli_sum;

/* Adjoint differentiation (Jones and Gacon, 2020) of <0|U^dag H U|0> with
 * U = U_G ... U_1 over the circuit's rotation angles, in the handle's dtype:
 *   psi = U|0>, phi = H psi, value = Re<psi|phi>; then for g = G..1:
 *   if gate g is exp(-i theta P/2): grad[param[g]] += Im<phi|P|psi>;
 *   psi <- U_g^dag psi; phi <- U_g^dag phi.
 * Uses three library-owned vectors of 2^n_qubits amplitudes (the handle's own
 * state is not touched).  grad_out has n_params entries.  Synchronises. */
qsv_status qsv_adjoint_gradient(qsv_sim *sim, const qsv_circuit *circ,
                                const qsv_pauli_sum *ham, double *value_out,
                                double *grad_out);

/* Batched expectation values: circuit b (gates only RX/RY/RZ/fixed matrices
 * on <= 2 qubits) and its Pauli sum give out[b] = <0|U_b^dag H_b U_b|0>.
 * A plan uploads the circuits once and holds an instantiated HIP graph of
 * its launches (a persistent launch for the circuits whose state fits in
 * LDS, pass-major launches for the larger ones); qsv_batch_run replays it. */
typedef struct qsv_batch qsv_batch;

typedef struct qsv_batch_options {
    int32_t dtype;            /* QSV_C64 or QSV_C128 */
    int32_t autotune;         /* 1: time candidate tile shapes on the first run */
    int32_t tile_bits;        /* 0 = default/autotuned */
    int32_t use_graph;        /* 1: capture the launch in a HIP graph */
    void *stream;
    const char *tune_cache;   /* JSON cache path, NULL = none */
    int32_t big_per_workgroup;/* circuits whose state exceeds the LDS tile: 0 (default) run
                                 pass-major, each state in its own device region, one launch
                                 per pass index over all their tiles, their Pauli sums in
                                 chunks (when the states fit in half the free device memory);
                                 1: each runs on one workgroup of the persistent launch */
} qsv_batch_options;

qsv_status qsv_batch_create(int32_t count, const qsv_circuit *circuits,
                            const qsv_pauli_sum *hams, const qsv_batch_options *opt,
                            qsv_batch **out);
qsv_status qsv_batch_run(qsv_batch *b, double *out_host);
/* Tile bits and fusion width in use (from the autotuner or the options) and
 * the device time of the last run in ms. */
qsv_status qsv_batch_info(const qsv_batch *b, int32_t *tile_bits, int32_t *k_fuse,
                          double *last_ms);
qsv_status qsv_batch_destroy(qsv_batch *b);

/* Message for the last failure on `sim` (or of the last qsv_create /
 * qsv_batch_* call when sim is NULL).  Valid until the next call. */
const char *qsv_last_error(const qsv_sim *sim);

const char *qsv_version(void);

/* Bandwidth probe: enqueue a streaming copy of `bytes` (a multiple of 16)
 * from device buffer src to device buffer dst on `stream` (a hipStream_t,
 * NULL = null stream).  Every state pass reads and writes the state once, so
 * this copy is the practical ceiling beside the HBM peak; timing it is the
 * caller's (HIP events on the same stream).  The buffers are the caller's and
 * must not overlap.  EINVAL: NULL buffer or bad size; EDEVICE: launch
 * failed (qsv_last_error(NULL) says why). */
qsv_status qsv_copy_probe(const void *src, void *dst, uint64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* QSV_H */
