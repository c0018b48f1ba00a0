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
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

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

Op relabel_op(const Op &o, const int *pos) {
    Op r = o;
    r.ctrl = 0;
    for (int p = 0; p < 64; ++p)
        if ((o.ctrl >> p) & 1) r.ctrl |= 1ull << pos[p];
    // new index bit i <- old index bit ord[i], targets ascending
    int ord[kMaxK];
    for (int j = 0; j < o.k; ++j) ord[j] = j;
    std::sort(ord, ord + o.k, [&](int a, int b) { return pos[o.t[a]] < pos[o.t[b]]; });
    for (int i = 0; i < o.k; ++i) r.t[i] = pos[o.t[ord[i]]];
    const int dim = 1 << o.k;
    auto beta = [&](int x) {
        int y = 0;
        for (int i = 0; i < o.k; ++i) y |= ((x >> ord[i]) & 1) << i;
        return y;
    };
    if (o.kind == Op::DENSE) {
        for (int row = 0; row < dim; ++row)
            for (int col = 0; col < dim; ++col)
                r.U[(size_t)beta(row) * dim + beta(col)] = o.U[(size_t)row * dim + col];
    } else {
        r.touch = 0;
        for (int row = 0; row < dim; ++row) {
            const int b = beta(row);
            r.perm[b] = (uint8_t)beta(o.perm[row]);
            r.U[b] = o.U[row];
            if ((o.touch >> row) & 1) r.touch |= 1u << b;
        }
    }
    return r;
}

std::vector<Pass> plan_passes_relabel(const std::vector<Op> &ops, int n, int m, int low_bits,
                                      int k_max, int kd_max, int page_bit, int page_cap,
                                      int op_cap) {
    std::vector<Pass> passes;
    if (ops.empty() || n <= m) return plan_passes(ops, n, m, low_bits, k_max, kd_max);
    const int L = std::max(0, std::min(low_bits, m - kMaxK));
    constexpr int kNever = 1 << 30;
    int pos[64], at[64];            // qubit -> position, position -> qubit
    for (int q = 0; q < 64; ++q) pos[q] = at[q] = q;
    std::vector<uint64_t> need(ops.size()), all(ops.size());
    for (size_t i = 0; i < ops.size(); ++i) {
        need[i] = ops[i].mixing();
        all[i] = ops[i].qubits();
    }
    auto page_qubits = [&]() {
        uint64_t pm = 0;
        for (int q = 0; q < n; ++q)
            if (pos[q] >= page_bit) pm |= 1ull << q;
        return pm;
    };
    auto to_positions = [&](uint64_t qmask) {
        uint64_t x = 0;
        for (int q = 0; q < n; ++q)
            if ((qmask >> q) & 1) x |= 1ull << pos[q];
        return x;
    };
    // Assign the qubits of `tile` (a mask of qubits) to the positions they
    // occupy, in the order given; record the moves as the pass's dest[].
    auto move = [&](Pass &ps, const std::vector<int> &qs_in_order, const std::vector<int> &home_first) {
        std::vector<int> slots;
        for (int q : qs_in_order) slots.push_back(pos[q]);
        for (int q : home_first) slots.push_back(pos[q]);
        std::sort(slots.begin(), slots.end());
        ps.dest.assign(n, 0);
        for (int p = 0; p < n; ++p) ps.dest[p] = (uint8_t)p;
        int np[64];
        for (int q = 0; q < n; ++q) np[q] = pos[q];
        std::vector<bool> taken(64, false);
        for (int q : home_first) {
            np[q] = q;
            taken[q] = true;
        }
        size_t k = 0;
        for (int q : qs_in_order) {
            while (taken[slots[k]]) ++k;
            np[q] = slots[k++];
        }
        for (int q = 0; q < n; ++q)
            if (np[q] != pos[q]) ps.dest[pos[q]] = (uint8_t)np[q];
        for (int q = 0; q < n; ++q) {
            pos[q] = np[q];
            at[np[q]] = q;
        }
    };
    std::vector<int> remaining(ops.size());
    for (size_t i = 0; i < ops.size(); ++i) remaining[i] = (int)i;
    while (!remaining.empty()) {
        const uint64_t pm = page_qubits();
        uint64_t low = 0;
        for (int p = 0; p < L; ++p) low |= 1ull << at[p];
        std::vector<int> in_pass, deferred;
        uint64_t tile = low;
        for (int cap : {page_cap, 64}) {
            tile = low;
            in_pass.clear();
            deferred.clear();
            uint64_t dmix = 0, dall = 0;
            for (int i : remaining) {
                const bool blocked = !commute_masks(dmix, dall, need[i], all[i]);
                const uint64_t t2 = tile | need[i];
                if (!blocked && popc(t2) <= m && popc(t2 & pm) <= cap &&
                    (int)in_pass.size() < op_cap) {
                    tile = t2;
                    in_pass.push_back(i);
                } else {
                    deferred.push_back(i);
                    dmix |= need[i];
                    dall |= all[i];
                }
            }
            if (!in_pass.empty()) break;
        }
        // Fill the tile up to m qubits: first with qubits that let a qubit
        // done for this flush go back to its own position (the qubit now at
        // a done qubit's own position, or a done qubit whose own position is
        // in the tile), while the tile stays within kFillPages page
        // positions; then with the qubits at the lowest positions.
        {
            uint64_t later = 0;
            for (int j : deferred) later |= all[j];
            auto tile_pages = [&](uint64_t t) {
                int h = 0;
                for (int q = 0; q < n; ++q)
                    if (((t >> q) & 1) && pos[q] >= page_bit) ++h;
                return h;
            };
            constexpr int kFillPages = 5;
            bool grew = true;
            while (grew && popc(tile) < m) {
                grew = false;
                for (int q = 0; q < n && popc(tile) < m; ++q) {
                    if (((later >> q) & 1) || pos[q] == q) continue;   // in use later, or home
                    const int r = at[q];                                // the qubit at q's position
                    uint64_t add = 0;
                    if (((tile >> q) & 1) && !((tile >> r) & 1)) add = 1ull << r;
                    else if (!((tile >> q) & 1) && ((tile >> r) & 1)) add = 1ull << q;
                    if (!add) continue;
                    const uint64_t t2 = tile | add;
                    if (tile_pages(t2) > std::max(kFillPages, tile_pages(tile))) continue;
                    tile = t2;
                    grew = true;
                }
            }
        }
        for (int p = 0; p < n && popc(tile) < m; ++p) tile |= 1ull << at[p];
        Pass ps;
        ps.tile = to_positions(tile);
        std::vector<Op> mapped;
        mapped.reserve(in_pass.size());
        for (int i : in_pass) mapped.push_back(relabel_op(ops[i], pos));
        ps.ops = fuse_impl(mapped, k_max, ps.tile, kd_max);
        // next use of each tile qubit among the deferred ops
        int next[64];
        for (int q = 0; q < 64; ++q) next[q] = kNever;
        uint64_t open = tile;
        for (int j = 0; j < (int)deferred.size() && open; ++j) {
            const uint64_t hit = open & need[deferred[j]];
            for (int q = 0; q < n; ++q)
                if ((hit >> q) & 1) next[q] = j;
            open &= ~hit;
        }
        // Qubits needed again soonest take the lowest positions (the ones
        // every tile holds, then those below the page bits); qubits done
        // for this flush go back to their own position when it is free.
        std::vector<int> order, home;
        for (int q = 0; q < n; ++q)
            if ((tile >> q) & 1) {
                if (next[q] == kNever && ((ps.tile >> q) & 1)) home.push_back(q);
                else order.push_back(q);
            }
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return next[a] < next[b]; });
        move(ps, order, home);
        passes.push_back(std::move(ps));
        remaining.swap(deferred);
    }
    // Restore the identity: follow the cycles of displaced qubits, each pass
    // sending home every qubit whose position is in its tile.
    for (;;) {
        int first = -1;
        for (int p = 0; p < n && first < 0; ++p)
            if (at[p] != p) first = p;
        if (first < 0) break;
        uint64_t S = (1ull << L) - 1;
        auto pages = [&](uint64_t x) { return popc(x >> page_bit); };
        for (int p0 = first; p0 < n && popc(S) < m; ++p0) {
            if (at[p0] == p0 || ((S >> p0) & 1)) continue;
            int p = p0;
            uint64_t add = 0;
            // p holds qubit at[p], whose own position is at[p]
            while (popc(S | add) < m) {
                if (!(((S | add) >> p) & 1)) add |= 1ull << p;
                const int nx = at[p];
                if (((S | add) >> nx) & 1) break;
                p = nx;
            }
            if (pages(S | add) > page_cap && S != ((1ull << L) - 1) && pages(S) < pages(S | add))
                continue;
            S |= add;
        }
        for (int p = 0; p < n && popc(S) < m; ++p) S |= 1ull << p;
        Pass ps;
        ps.tile = S;
        std::vector<int> order, home;
        for (int p = 0; p < n; ++p)
            if ((S >> p) & 1) {
                const int q = at[p];
                if ((S >> q) & 1) home.push_back(q);
                else order.push_back(q);
            }
        std::sort(order.begin(), order.end());
        move(ps, order, home);
        passes.push_back(std::move(ps));
    }
    return passes;
}

std::vector<Op> pass_ops_in_qubit_order(const std::vector<Pass> &passes, int n) {
    int qubit_at[64];
    for (int p = 0; p < 64; ++p) qubit_at[p] = p;
    std::vector<Op> out;
    for (const Pass &ps : passes) {
        for (const Op &o : ps.ops) out.push_back(relabel_op(o, qubit_at));
        if (ps.dest.empty()) continue;
        int nq[64];
        for (int p = 0; p < 64; ++p) nq[p] = qubit_at[p];
        for (int p = 0; p < n; ++p) nq[ps.dest[p]] = qubit_at[p];
        for (int p = 0; p < 64; ++p) qubit_at[p] = nq[p];
    }
    return out;
}

double plan_cost(const std::vector<Pass> &passes, int page_bit) {
    // relative time of a pass whose tile spans 2^h pages (measured on
    // 12-bit tiles of a 30-qubit complex128 state: flat up to 32 pages,
    // 1.2 x at 64, 2.3-4.7 x at 256), and of a pass that carries more fused
    // ops than its memory traffic hides (measured on the same tiles: a pass
    // reads and writes the state in about the time of 16 fused 2-qubit ops;
    // beyond that it grows with the ops; a diagonal op, one factor per
    // amplitude from a table, counts a quarter)
    static const double kCost[11] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.05, 1.2, 1.6, 2.5, 3.5, 4.7};
    constexpr double kOpsPerPass = 16.0;
    double c = 0.0;
    for (const Pass &p : passes) {
        double w = 0.0;
        for (const Op &o : p.ops) w += o.mixing() ? 1.0 : 0.25;
        c += kCost[std::min(10, popc(page_bit >= 64 ? 0 : p.tile >> page_bit))] *
             std::max(1.0, w / kOpsPerPass);
    }
    return c;
}

std::vector<Pass> plan_tiled(const std::vector<Op> &ops, int n, int m, int k_max, int page_bit,
                             bool relabel) {
    std::vector<Op> fused = fuse_impl(ops, k_max, ~0ull, kMaxK);
    std::vector<Pass> best = plan_passes(fused, n, m, 3, k_max, kMaxK);
    if (!relabel || n <= m) return best;
    // the greedy grouping reacts to the caps unevenly: plan with several page
    // caps and caps on the ops a pass takes, and keep the cheapest plan
    // (positions fixed included)
    // The candidates are independent: large queues plan them on several host
    // threads (the GPU waits for the plan), the choice is the same as in order.
    struct Cand {
        int op_cap, cap;
        std::vector<Pass> plan;
        double cost = 0.0;
    };
    std::vector<Cand> cands;
    for (int op_cap : {1 << 30, 40, 32})
        for (int cap : {2, 3, 4, 5, 8}) cands.push_back({op_cap, cap, {}, 0.0});
    auto work = [&](size_t i) {
        cands[i].plan = plan_passes_relabel(fused, n, m, 3, k_max, kMaxK, page_bit, cands[i].cap,
                                            cands[i].op_cap);
        cands[i].cost = plan_cost(cands[i].plan, page_bit);
    };
    const unsigned hw = std::thread::hardware_concurrency();
    const size_t nth = fused.size() < 64 ? 1 : std::min<size_t>(cands.size(), std::min(8u, std::max(1u, hw)));
    if (nth <= 1) {
        for (size_t i = 0; i < cands.size(); ++i) work(i);
    } else {
        std::atomic<size_t> next{0};
        std::vector<std::thread> th;
        th.reserve(nth);
        for (size_t t = 0; t < nth; ++t)
            th.emplace_back([&]() {
                for (size_t i; (i = next.fetch_add(1)) < cands.size();) work(i);
            });
        for (std::thread &x : th) x.join();
    }
    double best_cost = plan_cost(best, page_bit);
    for (Cand &c : cands)
        if (c.cost < best_cost - 1e-9) {
            best_cost = c.cost;
            best.swap(c.plan);
        }
    return best;
}
}  // namespace qsv
