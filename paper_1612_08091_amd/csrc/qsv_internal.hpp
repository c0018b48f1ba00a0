// Internal types shared by the planner, the C-ABI layer and the kernel
// launchers of libqsv.  Not part of the public interface.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace qsv {

using cd = std::complex<double>;

constexpr int kMaxK = 5;          // widest dense operation (32 x 32)
constexpr int kMaxQubits = 36;    // 2^36 c64 amplitudes = 512 GiB: beyond one GPU

inline int popc(uint64_t x) { return __builtin_popcountll(x); }

// One gate as queued: U (2^k x 2^k, row-major, bit j of the index <-> t[j])
// on bit positions t[0..k-1], applied where every bit of `ctrl` is 1.
struct Gate {
    int k = 0;
    int t[kMaxK] = {0, 0, 0, 0, 0};
    uint64_t ctrl = 0;
    std::vector<cd> U;
};

// A canonical operation.  DENSE: U is the full matrix.  MONO: one nonzero per
// row -- row r of the result takes val[r] * x[perm[r]]; rows outside `touch`
// are unchanged (perm[r] == r and val[r] == 1).  A MONO op with perm == id is
// diagonal.
struct Op {
    enum Kind { DENSE = 0, MONO = 1 };
    int kind = DENSE;
    int k = 0;
    int t[kMaxK] = {0, 0, 0, 0, 0};
    uint64_t ctrl = 0;
    bool diag = false;
    std::vector<cd> U;            // DENSE: 4^k entries; MONO: 2^k values
    uint8_t perm[32] = {};
    uint32_t touch = 0;
    int n_orig = 1;               // original gates merged into this op

    uint64_t targets() const {
        uint64_t m = 0;
        for (int j = 0; j < k; ++j) m |= 1ull << t[j];
        return m;
    }
    uint64_t qubits() const { return targets() | ctrl; }
    // Bit positions whose value the op may change.  Diagonal ops change none;
    // on every other qubit the op acts diagonally (controls, phases).
    uint64_t mixing() const { return diag ? 0 : targets(); }
};

// Diag-aware commutation test: two ops commute if on every shared qubit both
// act diagonally (sufficient, not necessary).
inline bool commute_masks(uint64_t mix_a, uint64_t all_a, uint64_t mix_b, uint64_t all_b) {
    uint64_t shared = all_a & all_b;
    return (shared & (mix_a | mix_b)) == 0;
}
inline bool commute(const Op &a, const Op &b) {
    return commute_masks(a.mixing(), a.qubits(), b.mixing(), b.qubits());
}

// Reduce a gate to canonical form: controls hidden inside the matrix are
// moved to `ctrl`, identity gates vanish (returns false), monomial matrices
// become MONO ops.
bool canonicalize(const Gate &g, Op &out);

// Greedy commutation-aware fusion into ops of at most k_max qubits (targets
// and controls together).  The fused matrices are products in complex128.
std::vector<Op> fuse(const std::vector<Op> &ops, int k_max);

// A pass over the state in LDS tiles: the 2^m amplitudes that share the
// values of the bits outside `tile` are processed together by one workgroup.
struct Pass {
    uint64_t tile = 0;            // bit positions inside a tile
    std::vector<Op> ops;
    // Relabeling: empty, or dest[p] = the position that the content of
    // position p (its qubit) occupies after the pass; a permutation of the
    // tile's positions, identity outside it.
    std::vector<uint8_t> dest;
};

// Greedy grouping behind the pass planner, on plain bit masks: item i needs
// the bits `need` inside the tile, changes the bits `mix` and touches `all`.
// Walking the remaining items in order, an item joins the current group if
// it commutes with every item deferred before it and its bits still fit in m
// (the lowest min(low_bits, m - kMaxK) positions are always in the tile);
// the group's tile is then filled up to m bits with the lowest free
// positions.  For n <= m there is one group holding everything.
struct PlanItem {
    uint64_t need = 0, mix = 0, all = 0;
};
struct PlanGroup {
    uint64_t tile = 0;
    std::vector<int> idx;         // item indices, in the order they are applied
};
std::vector<PlanGroup> plan_groups(const std::vector<PlanItem> &items, int n, int m,
                                   int low_bits);

// Group ops into passes whose mixing qubits fit in m tile bits, the lowest
// `low_bits` positions always included (contiguous HBM runs).  Ops are moved
// across each other only when they commute.  Then each pass is fused to
// k_max (only ops with all their qubits inside the tile are fused); runs of
// diagonal ops fuse into diagonal ops of up to kd_max qubits (at least k_max).
std::vector<Pass> plan_passes(const std::vector<Op> &ops, int n, int m, int low_bits,
                              int k_max, int kd_max = 0);

// The op with its qubit positions moved: position p -> pos[p] (controls and
// targets; targets come out ascending, the matrix permuted to match).
Op relabel_op(const Op &o, const int *pos);

// Pass planning with relabeling.  Every pass may also permute the positions
// of its tile (a permutation of where its qubits live, free in a pass that
// reads and writes the whole tile anyway).  Ops are planned on qubits; a pass
// takes its ops at the positions its qubits hold when it runs.  After each
// pass the qubits needed again soonest take the lowest tile positions: the
// `low_bits` positions present in every tile then hold useful qubits, and
// later tiles touch few positions at or above `page_bit` (one position there
// doubles the 2 MiB pages a tile spans).  Trailing passes without ops restore
// the identity, so the plan as a whole applies the ops and nothing else.
std::vector<Pass> plan_passes_relabel(const std::vector<Op> &ops, int n, int m, int low_bits,
                                      int k_max, int kd_max, int page_bit, int page_cap,
                                      int op_cap = 1 << 30);

// The ops of a plan in execution order, each on its qubits' own positions
// (the positions in effect when no pass relabels).
std::vector<Op> pass_ops_in_qubit_order(const std::vector<Pass> &passes, int n);

// Estimated time of a plan in passes over the state, each weighted by the
// number of 2 MiB pages its tile spans (a tile spread over 2^h pages reads
// far slower once h passes about 5) and by its ops beyond what its memory
// traffic hides (about 16 fused 2-qubit ops; a diagonal op counts a quarter).
double plan_cost(const std::vector<Pass> &passes, int page_bit);

// Whole-queue fusion to k_max first (diagonal runs to kMaxK qubits), then
// pass planning of the fused ops (blocks are not cut at pass boundaries);
// three low bits stay in every tile for contiguous HBM runs.  relabel: also
// plan with plan_passes_relabel under several page caps and caps on the ops
// per pass (none, 40, 32) and keep the plan of least plan_cost (page_bit: the amplitude index bit of a 2 MiB page, 17 for
// complex128 and 18 for complex64).
std::vector<Pass> plan_tiled(const std::vector<Op> &ops, int n, int m, int k_max,
                             int page_bit = 64, bool relabel = false);

// Dense 2^k x 2^k matrix of an op on its own target list (controls excluded).
std::vector<cd> dense_matrix(const Op &op);

// Message returned by qsv_last_error(NULL) (calls without a handle).
void set_last_error(const std::string &msg);

}  // namespace qsv
