// Host-side planning of a flush: gate canonicalisation, commutation-aware
// fusion into <= k_max-qubit unitaries (built in complex128), and grouping of
// operations into LDS-tile passes over the state.
//
// The paper attributes its simulator's speed to lazy evaluation of gates
// (Sec. 4.3.2): gates are cached and executed in bulk.  Fusion and pass
// planning are this library's way of exploiting that cache; they change the
// order of execution only across operations that commute, and they multiply
// matrices exactly (up to rounding), so the result is the per-gate result.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "qsv_internal.hpp"

namespace qsv {

namespace {

// Is U (dim x dim) the identity when restricted to the rows and columns with
// bit j = 0, with no coupling between bit j = 0 and bit j = 1?
bool bit_is_control(const std::vector<cd> &U, int k, int j) {
    const int dim = 1 << k;
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) {
            bool r0 = !((r >> j) & 1), c0 = !((c >> j) & 1);
            if (!r0 && !c0) continue;
            cd want = (r == c && r0) ? cd(1, 0) : cd(0, 0);
            if (U[(size_t)r * dim + c] != want) return false;
        }
    return true;
}

// Restrict U to bit j = 1 and drop bit j from the index.
std::vector<cd> drop_bit(const std::vector<cd> &U, int k, int j) {
    const int dim = 1 << k, nd = dim >> 1;
    std::vector<cd> out((size_t)nd * nd);
    auto up = [j](int x) { return ((x >> j) << (j + 1)) | (x & ((1 << j) - 1)) | (1 << j); };
    for (int r = 0; r < nd; ++r)
        for (int c = 0; c < nd; ++c) out[(size_t)r * nd + c] = U[(size_t)up(r) * dim + up(c)];
    return out;
}

// Apply op (acting on global bit positions) to every column of M, a
// 2^kb x 2^kb matrix over the block's positions `bq` (bit i of the block
// index <-> position bq[i]): M <- op * M.
void apply_op_to_block(std::vector<cd> &M, const std::vector<int> &bq, const Op &op) {
    const int kb = (int)bq.size();
    const int dim = 1 << kb;
    auto local_bit = [&](int pos) {
        for (int i = 0; i < kb; ++i)
            if (bq[i] == pos) return i;
        return -1;
    };
    int lt[kMaxK];
    for (int j = 0; j < op.k; ++j) lt[j] = local_bit(op.t[j]);
    uint32_t lctrl = 0;
    for (int p = 0; p < 64; ++p)
        if ((op.ctrl >> p) & 1) lctrl |= 1u << local_bit(p);
    const int od = 1 << op.k;
    std::vector<cd> U = dense_matrix(op);
    uint32_t tmask = 0;
    for (int j = 0; j < op.k; ++j) tmask |= 1u << lt[j];
    std::vector<cd> in(od), outv(od);
    for (int col = 0; col < dim; ++col) {
        for (int b = 0; b < dim; ++b) {
            if (b & tmask) continue;
            if ((b & lctrl) != lctrl) continue;
            for (int c = 0; c < od; ++c) {
                int idx = b;
                for (int j = 0; j < op.k; ++j)
                    if ((c >> j) & 1) idx |= 1 << lt[j];
                in[c] = M[(size_t)idx * dim + col];
            }
            for (int r = 0; r < od; ++r) {
                cd acc = 0;
                for (int c = 0; c < od; ++c) acc += U[(size_t)r * od + c] * in[c];
                outv[r] = acc;
            }
            for (int r = 0; r < od; ++r) {
                int idx = b;
                for (int j = 0; j < op.k; ++j)
                    if ((r >> j) & 1) idx |= 1 << lt[j];
                M[(size_t)idx * dim + col] = outv[r];
            }
        }
    }
}

bool make_mono(Op &op) {
    const int dim = 1 << op.k;
    uint8_t perm[32];
    cd val[32];
    bool col_used[32] = {};
    for (int r = 0; r < dim; ++r) {
        int nz = -1;
        for (int c = 0; c < dim; ++c)
            if (op.U[(size_t)r * dim + c] != cd(0, 0)) {
                if (nz >= 0) return false;
                nz = c;
            }
        if (nz < 0 || col_used[nz]) return false;
        col_used[nz] = true;
        perm[r] = (uint8_t)nz;
        val[r] = op.U[(size_t)r * dim + nz];
    }
    op.kind = Op::MONO;
    op.diag = true;
    op.touch = 0;
    op.U.assign(val, val + dim);
    for (int r = 0; r < dim; ++r) {
        op.perm[r] = perm[r];
        if (perm[r] != r) op.diag = false;
        if (perm[r] != r || val[r] != cd(1, 0)) op.touch |= 1u << r;
    }
    return true;
}

}  // namespace

std::vector<cd> dense_matrix(const Op &op) {
    if (op.kind == Op::DENSE) return op.U;
    const int dim = 1 << op.k;
    std::vector<cd> U((size_t)dim * dim, cd(0, 0));
    for (int r = 0; r < dim; ++r) U[(size_t)r * dim + op.perm[r]] = op.U[r];
    return U;
}

bool canonicalize(const Gate &g, Op &out) {
    Op op;
    op.kind = Op::DENSE;
    op.k = g.k;
    for (int j = 0; j < g.k; ++j) op.t[j] = g.t[j];
    op.ctrl = g.ctrl;
    op.U = g.U;
    // Controls hidden in the matrix become explicit controls (keep >= 1 target).
    bool changed = true;
    while (changed && op.k > 1) {
        changed = false;
        for (int j = 0; j < op.k; ++j) {
            if (bit_is_control(op.U, op.k, j)) {
                op.U = drop_bit(op.U, op.k, j);
                op.ctrl |= 1ull << op.t[j];
                for (int i = j; i + 1 < op.k; ++i) op.t[i] = op.t[i + 1];
                op.k -= 1;
                changed = true;
                break;
            }
        }
    }
    if (op.k == 1 && bit_is_control(op.U, 1, 0) && op.U[3] == cd(1, 0)) return false;  // identity
    if (make_mono(op) && op.touch == 0) return false;                                  // identity
    out = std::move(op);
    return true;
}

// ---------------------------------------------------------------- fusion
namespace {

struct Block {
    uint64_t all = 0, mix = 0;
    bool diag = true;            // every member is diagonal
    std::vector<int> members;
};

Op build_block(const std::vector<Op> &ops, const Block &b) {
    if (b.members.size() == 1) return ops[b.members[0]];
    std::vector<int> bq;
    for (int p = 0; p < 64; ++p)
        if ((b.all >> p) & 1) bq.push_back(p);
    const int kb = (int)bq.size();
    const int dim = 1 << kb;
    std::vector<cd> M((size_t)dim * dim, cd(0, 0));
    for (int i = 0; i < dim; ++i) M[(size_t)i * dim + i] = 1;
    int norig = 0;
    for (int m : b.members) {
        apply_op_to_block(M, bq, ops[m]);
        norig += ops[m].n_orig;
    }
    Gate g;
    g.k = kb;
    for (int i = 0; i < kb; ++i) g.t[i] = bq[i];
    g.ctrl = 0;
    g.U = std::move(M);
    Op out;
    if (!canonicalize(g, out)) {
        // The product is the identity: keep a trivial diagonal op so the
        // original-gate count is preserved; it touches nothing.
        out = Op();
        out.kind = Op::MONO;
        out.k = 1;
        out.t[0] = bq[0];
        out.diag = true;
        out.U = {cd(1, 0), cd(1, 0)};
        out.perm[0] = 0;
        out.perm[1] = 1;
        out.touch = 0;
    }
    out.n_orig = norig;
    return out;
}

// kd_max: a diagonal op fuses with a diagonal block it shares a qubit with up
// to kd_max qubits (a run of phases stays one diagonal op, cheap to apply);
// every other block stays within k_max.
std::vector<Op> fuse_impl(const std::vector<Op> &ops, int k_max, uint64_t allowed, int kd_max) {
    std::vector<Block> blocks;
    std::vector<bool> frozen;   // blocks that may not absorb anything
    kd_max = std::max(kd_max, k_max);
    for (int i = 0; i < (int)ops.size(); ++i) {
        const Op &op = ops[i];
        const uint64_t all = op.qubits(), mix = op.mixing();
        const bool dg = op.kind == Op::MONO && op.diag;
        const bool fusable =
            k_max >= 1 && (all & ~allowed) == 0 && popc(all) <= (dg ? kd_max : k_max);
        // latest block that does not commute with op
        int j = -1;
        for (int b = (int)blocks.size() - 1; b >= 0; --b)
            if (!commute_masks(blocks[b].mix, blocks[b].all, mix, all)) { j = b; break; }
        int best = -1, best_ov = -1;
        if (fusable) {
            for (int b = std::max(j, 0); b < (int)blocks.size(); ++b) {
                if (frozen[b]) continue;
                const int ov = popc(blocks[b].all & all);
                // a diagonal block grows past k_max only along shared qubits
                // (a chain of phases on one qubit), so unrelated phases stay
                // free to fuse with the dense gates next to them
                const int lim = (dg && blocks[b].diag && ov > 0) ? kd_max : k_max;
                if (popc(blocks[b].all | all) > lim) continue;
                if (ov >= best_ov) { best = b; best_ov = ov; }
            }
        }
        if (best >= 0) {
            blocks[best].all |= all;
            blocks[best].mix |= mix;
            blocks[best].diag = blocks[best].diag && dg;
            blocks[best].members.push_back(i);
        } else {
            Block nb;
            nb.all = all;
            nb.mix = mix;
            nb.diag = dg;
            nb.members.push_back(i);
            blocks.push_back(nb);
            frozen.push_back(!fusable);
        }
    }
    std::vector<Op> out;
    out.reserve(blocks.size());
    for (const Block &b : blocks) out.push_back(build_block(ops, b));
    return out;
}

}  // namespace

std::vector<Op> fuse(const std::vector<Op> &ops, int k_max) {
    return fuse_impl(ops, k_max, ~0ull, k_max);
}

// ---------------------------------------------------------- pass planning
std::vector<PlanGroup> plan_groups(const std::vector<PlanItem> &items, int n, int m,
                                   int low_bits) {
    std::vector<PlanGroup> groups;
    if (items.empty()) return groups;
    const uint64_t all_bits = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    if (n <= m) {
        PlanGroup g;
        g.tile = all_bits;
        for (int i = 0; i < (int)items.size(); ++i) g.idx.push_back(i);
        groups.push_back(std::move(g));
        return groups;
    }
    const int L = std::max(0, std::min(low_bits, m - kMaxK));
    const uint64_t low = (1ull << L) - 1;
    std::vector<int> remaining(items.size());
    for (int i = 0; i < (int)items.size(); ++i) remaining[i] = i;
    while (!remaining.empty()) {
        uint64_t tile = low;
        std::vector<int> in_pass, deferred;
        uint64_t dmix = 0, dall = 0;
        for (int i : remaining) {
            const PlanItem &it = items[i];
            const bool blocked = !commute_masks(dmix, dall, it.mix, it.all);
            if (!blocked && popc(tile | it.need) <= m) {
                tile |= it.need;
                in_pass.push_back(i);
            } else {
                deferred.push_back(i);
                dmix |= it.mix;
                dall |= it.all;
            }
        }
        // Fill the tile up to m bits with the lowest free positions.
        for (int p = 0; p < n && popc(tile) < m; ++p) tile |= 1ull << p;
        PlanGroup g;
        g.tile = tile;
        g.idx = std::move(in_pass);
        groups.push_back(std::move(g));
        remaining.swap(deferred);
    }
    return groups;
}

std::vector<Pass> plan_passes(const std::vector<Op> &ops, int n, int m, int low_bits,
                              int k_max, int kd_max) {
    std::vector<PlanItem> items(ops.size());
    for (size_t i = 0; i < ops.size(); ++i) {
        items[i].need = items[i].mix = ops[i].mixing();
        items[i].all = ops[i].qubits();
    }
    std::vector<Pass> passes;
    for (const PlanGroup &g : plan_groups(items, n, m, low_bits)) {
        std::vector<Op> in_pass;
        in_pass.reserve(g.idx.size());
        for (int i : g.idx) in_pass.push_back(ops[i]);
        Pass ps;
        ps.tile = g.tile;
        ps.ops = fuse_impl(in_pass, k_max, g.tile, kd_max);
        passes.push_back(std::move(ps));
    }
    return passes;
}

}  // namespace qsv

namespace qsv {
std::vector<Pass> plan_tiled(const std::vector<Op> &ops, int n, int m, int k_max) {
    return plan_passes(fuse_impl(ops, k_max, ~0ull, kMaxK), n, m, 3, k_max, kMaxK);
}
}  // namespace qsv
