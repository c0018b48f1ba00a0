// Lowering of a planned pass into the instruction list of a tile kernel.
//
// For the register-resident kernel (m = RB + 8 tile bits, 2^RB amplitudes per
// thread) this decides, op by op, which tile bits live in registers: a 1- or
// 2-qubit dense operation needs its targets there; when it finds them absent
// a REMAP moves the tile through LDS into a layout holding the targets plus
// the bits used soonest afterwards (Belady's furthest-next-use rule applied
// to the RB register slots).  Diagonal operations run in any layout; wider
// operations run on the LDS copy of the tile.
#include <algorithm>
#include <cstring>

#include "device.hpp"
#include "qsv_internal.hpp"
#include "tileprog.hpp"

namespace qsv {

uint32_t swz_elem(uint32_t l, int elem_bytes) {
    return elem_bytes == 16 ? (l ^ (((l >> 4) ^ (l >> 8)) & 15u))
                            : (l ^ (((l >> 5) ^ (l >> 10)) & 31u));
}

namespace {

void push(std::vector<double> &mats, const cd &v) {
    mats.push_back(v.real());
    mats.push_back(v.imag());
}

// TileOp (LDS kernel form) of an op whose mixing targets lie in the tile;
// li maps global positions to local bits, m = number of tile bits.
dev::TileOp lds_form(const Op &op, const int *li, std::vector<double> &mats, int elem_bytes,
                     double *flops) {
    dev::TileOp t{};
    t.k = op.k;
    t.touch = op.touch;
    t.mat = (int64_t)(mats.size() / 2);
    int m = 0;
    for (int p = 0; p < 64; ++p)
        if (li[p] >= 0) ++m;
    bool inside = true;
    for (int j = 0; j < op.k; ++j)
        if (li[op.t[j]] < 0) inside = false;
    // diagonal ops of more than three targets, or with targets outside the
    // tile, take their phase index from the global index of each amplitude
    if (op.kind == Op::MONO && op.diag && (!inside || op.k > 3)) {
        t.kind = dev::TOP_DIAG_GLOBAL;
        for (int j = 0; j < op.k; ++j) t.gt[j] = (uint32_t)op.t[j];
        t.gctrl = op.ctrl;
        for (int r = 0; r < (1 << op.k); ++r) push(mats, op.U[r]);
        *flops = 6.0 * __builtin_popcount(op.touch) / (double)(1 << op.k) /
                 (double)(1ull << popc(op.ctrl));
        return t;
    }
    // monomial ops of 4 or more qubits run as dense (matrix-core) ops, which
    // keeps the per-thread register arrays of the LDS kernel small
    const bool mono = op.kind == Op::MONO && op.k <= 3;
    t.kind = mono ? dev::TOP_MONO : dev::TOP_DENSE;
    uint32_t lctrl = 0;
    uint64_t ectrl = 0;
    for (int p = 0; p < 64; ++p)
        if ((op.ctrl >> p) & 1) {
            if (li[p] >= 0) lctrl |= 1u << li[p];
            else ectrl |= 1ull << p;
        }
    t.ectrl = ectrl;
    uint32_t ins = lctrl;
    int lt[kMaxK];
    for (int j = 0; j < op.k; ++j) {
        lt[j] = li[op.t[j]];
        ins |= 1u << lt[j];
    }
    t.nfree = 0;
    for (int b = 0; b < m; ++b)
        if (!((ins >> b) & 1)) t.fz[t.nfree++] = swz_elem(1u << b, elem_bytes) * elem_bytes;
    for (int r = 0; r < (1 << op.k); ++r) {
        uint32_t o = 0;
        for (int j = 0; j < op.k; ++j)
            if ((r >> j) & 1) o |= 1u << lt[j];
        t.sl[r] = swz_elem(o | lctrl, elem_bytes) * elem_bytes;
    }
    const double frac = 1.0 / (double)(1ull << popc(op.ctrl));
    if (mono) {
        for (int r = 0; r < (1 << op.k); ++r) {
            t.ss[r] = t.sl[op.perm[r]];
            push(mats, op.U[r]);
        }
        *flops = frac * 6.0 * __builtin_popcount(op.touch) / (double)(1 << op.k);
    } else if (op.k >= 3) {
        // matrix cores: real embedding W = [[Re U, -Im U], [Im U, Re U]],
        // stored in the order the 16x16x4 A operand is read: fragment
        // (mb, kc) is 64 consecutive values, lane l holding
        // W[16 mb + l % 16][4 kc + l / 16], so each fragment load is one
        // contiguous read across the wave.  The pool is in complex entries;
        // the fragments take 2 D * 2 D reals = 2 D^2 complex slots.
        t.kind = dev::TOP_DENSE_MFMA;
        const int D = 1 << op.k, D2 = 2 * D, MB = D2 / 16, KC = D2 / 4;
        const std::vector<cd> U = dense_matrix(op);
        auto w_at = [&](int i, int j) {
            const cd u = U[(size_t)(i % D) * D + (j % D)];
            if (i < D) return (j < D) ? u.real() : -u.imag();
            return (j < D) ? u.imag() : u.real();
        };
        for (int mb = 0; mb < MB; ++mb)
            for (int kc = 0; kc < KC; ++kc)
                for (int l = 0; l < 64; ++l) mats.push_back(w_at(16 * mb + l % 16, 4 * kc + l / 16));
        *flops = frac * (8.0 * D - 2.0);
    } else {
        for (const cd &v : dense_matrix(op)) push(mats, v);
        *flops = frac * (8.0 * (1 << op.k) - 2.0);
    }
    return t;
}

void set_layout(uint32_t regmask, int m, int rb, uint8_t *reg_lbit, uint8_t *thr_lbit) {
    int j = 0, i = 0;
    for (int b = 0; b < m; ++b) {
        if ((regmask >> b) & 1) reg_lbit[j++] = (uint8_t)b;
        else thr_lbit[i++] = (uint8_t)b;
    }
    (void)rb;
}

}  // namespace

uint32_t remap_offset(uint32_t l, int kept, int elem_bytes) {
    const uint32_t lowm = (1u << kept) - 1;
    const uint32_t h = ((l >> 1) & ~lowm) | (l & lowm);
    return swz_elem(h, elem_bytes) * (uint32_t)elem_bytes;
}

namespace {

// Global-index bits and LDS byte offsets of every layout of a register
// program (the kernel then needs no per-lane layout arithmetic).
void fill_layouts(TileProgram &prog, int rb, int elem_bytes) {
    uint8_t tpos[64];
    int c = 0;
    for (int p = 0; p < 64; ++p)
        if ((prog.tile >> p) & 1) tpos[c++] = (uint8_t)p;
    const int tb = prog.m - rb;
    const int nr = 1 << rb;
    for (int j = 0; j < rb; ++j) prog.g_reg[j] = 1ull << tpos[prog.reg_lbit[j]];
    for (int t = 0; t < tb; ++t) prog.g_thr[t] = 1ull << tpos[prog.thr_lbit[t]];
    uint8_t cur_reg[8], cur_thr[16];
    std::memcpy(cur_reg, prog.reg_lbit, 8);
    std::memcpy(cur_thr, prog.thr_lbit, 16);
    for (dev::RegOp &r : prog.rops) {
        if (r.kind != dev::ROP_REMAP) continue;
        const int kept = cur_reg[r.a];
        for (int i = 0; i < nr; ++i) {
            uint32_t lo = 0, ln = 0;
            for (int j = 0; j < rb; ++j)
                if ((i >> j) & 1) {
                    lo |= 1u << cur_reg[j];
                    ln |= 1u << r.reg_lbit[j];
                }
            r.wr[i] = remap_offset(lo, kept, elem_bytes);
            r.rd[i] = remap_offset(ln, kept, elem_bytes);
        }
        for (int t = 0; t < tb; ++t) {
            r.wthr[t] = remap_offset(1u << cur_thr[t], kept, elem_bytes);
            r.rthr[t] = remap_offset(1u << r.thr_lbit[t], kept, elem_bytes);
            r.g_thr[t] = 1ull << tpos[r.thr_lbit[t]];
        }
        for (int j = 0; j < rb; ++j) r.g_reg[j] = 1ull << tpos[r.reg_lbit[j]];
        std::memcpy(cur_reg, r.reg_lbit, 8);
        std::memcpy(cur_thr, r.thr_lbit, 16);
    }
}

}  // namespace

void compile_pass(const Pass &ps, int rb, std::vector<double> &mats, TileProgram &prog,
                  int elem_bytes) {
    prog = TileProgram();
    prog.tile = ps.tile;
    int li[64];
    int m = 0;
    for (int p = 0; p < 64; ++p) {
        li[p] = -1;
        if ((ps.tile >> p) & 1) li[p] = m++;
    }
    prog.m = m;
    const int tb = m - rb;
    prog.reg = rb >= 3 && rb <= 5 && (tb == 8 || (tb == 9 && rb <= 4));
    // the register kernel runs 1- and 2-qubit dense ops and diagonal ops only
    for (const Op &op : ps.ops) {
        if (op.kind == Op::MONO && (op.diag || op.touch == 0)) continue;
        bool inside = true;
        for (int j = 0; j < op.k; ++j)
            if (li[op.t[j]] < 0) inside = false;
        if (!inside || op.k > 2) prog.reg = false;
    }
    if (!prog.reg) {
        for (const Op &op : ps.ops) {
            if (op.kind == Op::MONO && op.touch == 0) continue;
            double fl = 0.0;
            dev::TileOp t = lds_form(op, li, mats, elem_bytes, &fl);
            prog.flops_per_amp += fl;
            if (t.kind == dev::TOP_DENSE_MFMA) prog.mfma_k = std::max(prog.mfma_k, t.k);
            prog.lops.push_back(t);
        }
        return;
    }
    // classify
    struct Item {
        int kind;          // ROP_G1/G2/DIAG/LDS
        uint32_t need;     // local bits that must be register bits
        const Op *op;
        int run;           // DIAG: index into `runs`
    };
    // A run of consecutive diagonal ops becomes one diagonal op: the controls
    // that all of them share stay controls, every other qubit of the run
    // (targets and the remaining controls) indexes the table, while there are
    // at most kRegDiagMax such qubits.  The kernel's cost of a diagonal op is
    // one table gather and one complex product per amplitude, whatever its
    // width.  A run of one op keeps its own targets and controls.
    struct DiagRun {
        int k = 0;
        int t[dev::kRegDiagMax] = {};
        uint64_t ctrl = 0;
        std::vector<cd> val;   // val[r], bit j of r <-> qubit t[j]
    };
    std::vector<DiagRun> runs;
    std::vector<uint64_t> run_all;   // qubits of each run (for commutation)
    std::vector<Item> items;
    const int n_ops = (int)ps.ops.size();
    auto is_diag = [](const Op &o) { return o.kind == Op::MONO && o.diag && o.touch != 0; };
    auto is_noop = [](const Op &o) { return o.kind == Op::MONO && o.touch == 0; };
    for (int oi = 0; oi < n_ops; ++oi) {
        const Op &op = ps.ops[oi];
        if (is_noop(op)) continue;
        if (is_diag(op)) {
            uint64_t common = op.ctrl, qs = op.targets();
            std::vector<const Op *> mem{&op};
            int oj = oi + 1;
            for (; oj < n_ops; ++oj) {
                const Op &o2 = ps.ops[oj];
                if (is_noop(o2)) continue;
                if (!is_diag(o2)) break;
                const uint64_t c2 = common & o2.ctrl;
                const uint64_t q2 = qs | (common & ~c2) | (o2.qubits() & ~c2);
                if (popc(q2) > dev::kRegDiagMax) break;
                common = c2;
                qs = q2;
                mem.push_back(&o2);
            }
            DiagRun run;
            if (mem.size() == 1) {
                run.k = op.k;
                for (int j = 0; j < op.k; ++j) run.t[j] = op.t[j];
                run.ctrl = op.ctrl;
                run.val.assign(op.U.begin(), op.U.begin() + (1 << op.k));
            } else {
                run.ctrl = common;
                for (int p = 0; p < 64; ++p)
                    if ((qs >> p) & 1) run.t[run.k++] = p;
                run.val.assign(size_t(1) << run.k, cd(1, 0));
                for (uint32_t r = 0; r < (1u << run.k); ++r) {
                    uint64_t bits = common;   // the qubits' values in row r
                    for (int j = 0; j < run.k; ++j)
                        if ((r >> j) & 1) bits |= 1ull << run.t[j];
                    for (const Op *o : mem) {
                        if ((bits & o->ctrl) != o->ctrl) continue;
                        uint32_t row = 0;
                        for (int j = 0; j < o->k; ++j)
                            if ((bits >> o->t[j]) & 1) row |= 1u << j;
                        run.val[r] *= o->U[row];
                    }
                }
                prog.diag_merged += (int)mem.size() - 1;
            }
            uint64_t all = 0;
            for (const Op *o : mem) all |= o->qubits();
            run_all.push_back(all);
            runs.push_back(std::move(run));
            items.push_back({dev::ROP_DIAG, 0u, nullptr, (int)runs.size() - 1});
            oi = oj - 1;
            continue;
        }
        bool inside = true;
        uint32_t need = 0;
        for (int j = 0; j < op.k; ++j) {
            if (li[op.t[j]] < 0) inside = false;
            else need |= 1u << li[op.t[j]];
        }
        if (inside && op.k <= 2) items.push_back({op.k == 1 ? dev::ROP_G1 : dev::ROP_G2, need, &op, -1});
        else items.push_back({dev::ROP_LDS, 0u, &op, -1});
    }
    // Ops of a pass that commute may run in any order.  List scheduling over
    // the order that non-commuting ops impose: among the ops whose
    // predecessors have run, take the first (in queue order) whose bits are
    // already register bits; if none is, the one with the fewest bits missing
    // (its layout change keeps more of the register set that the waiting ops
    // may want, and every change is a workgroup-wide LDS round trip), and
    // model the new register set as its bits plus the old register bits that
    // the most waiting ops need.  The lowering below then places the layout
    // changes.  The choice is among the next kWin unscheduled ops (queue
    // order), which bounds the cost on long passes: the first unscheduled op
    // is always ready, and an op further than kWin behind an unscheduled
    // one cannot be picked, so only dependences within kWin need recording.
    {
        constexpr int kWin = 256;
        const int N = (int)items.size();
        std::vector<uint64_t> q_all(N), q_mix(N);
        for (int i = 0; i < N; ++i) {
            if (items[i].run >= 0) {
                q_all[i] = run_all[items[i].run];
                q_mix[i] = 0;
            } else {
                q_all[i] = items[i].op->qubits();
                q_mix[i] = items[i].op->mixing();
            }
        }
        std::vector<int> npred(N, 0);
        std::vector<std::vector<int>> succ(N);
        for (int i = 0; i < N; ++i)
            for (int j = std::max(0, i - kWin); j < i; ++j)
                if (!commute_masks(q_mix[j], q_all[j], q_mix[i], q_all[i])) {
                    succ[j].push_back(i);
                    npred[i] += 1;
                }
        uint32_t Sm = 0;
        for (const Item &it : items) {
            if (__builtin_popcount(Sm | it.need) > rb) break;
            Sm |= it.need;
        }
        std::vector<char> ready(N, 0), done(N, 0);
        for (int i = 0; i < N; ++i) ready[i] = npred[i] == 0;
        std::vector<Item> order;
        order.reserve(N);
        int first = 0;   // first unscheduled op
        for (int step = 0; step < N; ++step) {
            while (done[first]) ++first;
            const int end = std::min(N, first + kWin);
            int pick = -1;
            for (int i = first; i < end && pick < 0; ++i)
                if (ready[i] && !done[i] && (items[i].need & ~Sm) == 0) pick = i;
            if (pick < 0) {
                int fewest = 1 << 30;
                for (int i = first; i < end; ++i)
                    if (ready[i] && !done[i]) {
                        const int miss = __builtin_popcount(items[i].need & ~Sm);
                        if (miss < fewest) {
                            fewest = miss;
                            pick = i;
                        }
                    }
                // new register set: the op's bits, then the old register bits
                // wanted by the most ops that wait (ready ones count more)
                uint32_t Sn = items[pick].need;
                int cnt[32] = {0};
                for (int i = first; i < end; ++i)
                    if (!done[i] && i != pick)
                        for (int b = 0; b < m; ++b)
                            if ((items[i].need >> b) & 1) cnt[b] += ready[i] ? 4 : 1;
                while (__builtin_popcount(Sn) < rb) {
                    int best = -1;
                    for (int b = 0; b < m; ++b)
                        if (!((Sn >> b) & 1) && ((Sm >> b) & 1) && (best < 0 || cnt[b] > cnt[best]))
                            best = b;
                    if (best < 0) break;
                    Sn |= 1u << best;
                }
                Sm = Sn;
            }
            done[pick] = 1;
            order.push_back(items[pick]);
            for (int j : succ[pick])
                if (--npred[j] == 0) ready[j] = 1;
        }
        items.swap(order);
    }
    const int n_items = (int)items.size();
    // next_at[i * m + b]: the first op at or after position i that needs
    // tile bit b (1 << 30: none), for the Belady choices of the remaps
    std::vector<int> next_at((size_t)(n_items + 1) * m, 1 << 30);
    for (int i = n_items - 1; i >= 0; --i)
        for (int b = 0; b < m; ++b)
            next_at[(size_t)i * m + b] =
                ((items[i].need >> b) & 1) ? i : next_at[(size_t)(i + 1) * m + b];
    // initial register set: the first needed bits, then the highest free bits
    uint32_t S = 0;
    for (const Item &it : items) {
        if (__builtin_popcount(S | it.need) > rb) break;
        S |= it.need;
        if (__builtin_popcount(S) == rb) break;
    }
    for (int b = m - 1; b >= 0 && __builtin_popcount(S) < rb; --b) S |= 1u << b;
    set_layout(S, m, rb, prog.reg_lbit, prog.thr_lbit);
    uint8_t cur_reg[8], cur_thr[16];
    std::memcpy(cur_reg, prog.reg_lbit, 8);
    std::memcpy(cur_thr, prog.thr_lbit, 16);

    for (int i = 0; i < n_items; ++i) {
        const Item &it = items[i];
        if ((it.need & ~S) != 0) {
            int next_use[32];
            for (int b = 0; b < m; ++b) next_use[b] = next_at[(size_t)i * m + b];
            uint32_t Sn = it.need;
            std::vector<int> cand;
            for (int b = 0; b < m; ++b)
                if (!((Sn >> b) & 1)) cand.push_back(b);
            std::sort(cand.begin(), cand.end(), [&](int x, int y) {
                if (next_use[x] != next_use[y]) return next_use[x] < next_use[y];
                const bool sx = (S >> x) & 1, sy = (S >> y) & 1;
                if (sx != sy) return sx;
                return x > y;
            });
            for (int c = 0; c < (int)cand.size() && __builtin_popcount(Sn) < rb; ++c)
                Sn |= 1u << cand[c];
            // The two-phase remap needs one tile bit that stays in its register
            // slot: keep the old register bit used soonest if none survived.
            if ((Sn & S) == 0) {
                int keep = -1, drop = -1;
                for (int b = 0; b < m; ++b)
                    if (((S >> b) & 1) && (keep < 0 || next_use[b] < next_use[keep])) keep = b;
                for (int b = 0; b < m; ++b)
                    if (((Sn >> b) & 1) && !((it.need >> b) & 1) &&
                        (drop < 0 || next_use[b] > next_use[drop]))
                        drop = b;
                Sn = (Sn & ~(1u << drop)) | (1u << keep);
            }
            int split = -1;   // slot of the surviving bit (soonest used)
            for (int j = 0; j < rb; ++j)
                if (((Sn >> cur_reg[j]) & 1) &&
                    (split < 0 || next_use[cur_reg[j]] < next_use[cur_reg[split]]))
                    split = j;
            dev::RegOp r{};
            r.kind = dev::ROP_REMAP;
            r.a = split;
            set_layout(Sn, m, rb, r.reg_lbit, r.thr_lbit);
            // put the surviving bit back into its slot
            for (int j = 0; j < rb; ++j)
                if (r.reg_lbit[j] == cur_reg[split]) std::swap(r.reg_lbit[j], r.reg_lbit[split]);
            std::memcpy(cur_reg, r.reg_lbit, 8);
            std::memcpy(cur_thr, r.thr_lbit, 16);
            prog.rops.push_back(r);
            prog.remaps += 1;
            S = Sn;
        }
        dev::RegOp r{};
        r.kind = it.kind;
        if (it.kind == dev::ROP_DIAG) {
            // split the row index and the controls into register bits (wr[i]
            // per register index i, b) and the rest (pad0, ctrl)
            auto reg_of = [&](int pos) {
                for (int j = 0; j < rb; ++j)
                    if (li[pos] >= 0 && cur_reg[j] == li[pos]) return j;
                return -1;
            };
            const DiagRun &run = runs[it.run];
            r.a = run.k;
            r.pad0 = 0;
            for (int j = 0; j < run.k; ++j) {
                r.gt[j] = (uint32_t)run.t[j];
                const int rj = reg_of(run.t[j]);
                if (rj < 0) r.pad0 |= 1u << j;
                for (int i = 0; i < (1 << rb); ++i)
                    if (rj >= 0 && ((i >> rj) & 1)) r.wr[i] |= 1u << j;
            }
            r.ctrl = 0;
            r.b = 0;
            for (int p = 0; p < 64; ++p)
                if ((run.ctrl >> p) & 1) {
                    const int rj = reg_of(p);
                    if (rj >= 0) r.b |= 1 << rj;
                    else r.ctrl |= 1ull << p;
                }
            r.mat = (int64_t)(mats.size() / 2);
            int changed = 0;
            for (int e = 0; e < (1 << run.k); ++e) {
                push(mats, run.val[e]);
                if (run.val[e] != cd(1, 0)) ++changed;
            }
            prog.flops_per_amp += 6.0 * changed / (double)(1 << run.k) /
                                  (double)(1ull << popc(run.ctrl));
        } else if (it.kind == dev::ROP_LDS) {
            const Op &op = *it.op;
            double fl = 0.0;
            dev::TileOp t = lds_form(op, li, mats, elem_bytes, &fl);
            prog.flops_per_amp += fl;
            r.a = (int32_t)prog.lops.size();
            prog.lops.push_back(t);
        } else {
            const Op &op = *it.op;
            auto reg_index = [&](int local_bit) {
                for (int j = 0; j < rb; ++j)
                    if (cur_reg[j] == local_bit) return j;
                return -1;
            };
            std::vector<cd> U = dense_matrix(op);
            r.ctrl = op.ctrl;
            r.mat = (int64_t)(mats.size() / 2);
            if (it.kind == dev::ROP_G1) {
                r.a = reg_index(li[op.t[0]]);
                for (const cd &v : U) push(mats, v);
                prog.flops_per_amp += 14.0 / (double)(1ull << popc(op.ctrl));
            } else {
                const int j0 = reg_index(li[op.t[0]]), j1 = reg_index(li[op.t[1]]);
                if (j0 < j1) {
                    r.a = j0;
                    r.b = j1;
                    for (const cd &v : U) push(mats, v);
                } else {
                    r.a = j1;
                    r.b = j0;
                    auto sw = [](int x) { return ((x & 1) << 1) | ((x >> 1) & 1); };
                    for (int row = 0; row < 4; ++row)
                        for (int col = 0; col < 4; ++col) push(mats, U[sw(row) * 4 + sw(col)]);
                }
                prog.flops_per_amp += 30.0 / (double)(1ull << popc(op.ctrl));
            }
        }
        prog.rops.push_back(r);
    }
    // Stores leave from the final layout.  With some of the three lowest tile
    // bits in registers and the first two thread bits far up the index, each
    // store instruction writes 16-byte pieces of many separate 128-byte
    // lines, and the memory system writes them out more than once (measured:
    // 2.5 x the state for one pass of the 30-qubit brick circuit).  A final
    // remap to a layout without those bits in registers costs less.
    if (S & 0x7u) {
        int gpos[32], c = 0;
        for (int p = 0; p < 64; ++p)
            if ((ps.tile >> p) & 1) gpos[c++] = p;
        if (tb >= 2 && (gpos[cur_thr[0]] > 5 || gpos[cur_thr[1]] > 6)) {
            uint32_t Sn = S & ~0x7u;
            for (int b = m - 1; b >= 3 && __builtin_popcount(Sn) < rb; --b) Sn |= 1u << b;
            int split = -1;
            for (int j = 0; j < rb && split < 0; ++j)
                if ((Sn >> cur_reg[j]) & 1) split = j;
            if (split >= 0 && __builtin_popcount(Sn) == rb) {
                dev::RegOp r{};
                r.kind = dev::ROP_REMAP;
                r.a = split;
                set_layout(Sn, m, rb, r.reg_lbit, r.thr_lbit);
                for (int j = 0; j < rb; ++j)
                    if (r.reg_lbit[j] == cur_reg[split]) std::swap(r.reg_lbit[j], r.reg_lbit[split]);
                std::memcpy(cur_reg, r.reg_lbit, 8);
                std::memcpy(cur_thr, r.thr_lbit, 16);
                prog.rops.push_back(r);
                prog.remaps += 1;
                S = Sn;
            }
        }
    }
    fill_layouts(prog, rb, elem_bytes);
    // the kernel runs ops in pairs: pad with an identity 1-qubit op
    if (prog.rops.size() & 1) {
        dev::RegOp nop{};
        nop.kind = dev::ROP_G1;
        nop.a = 0;
        nop.mat = (int64_t)(mats.size() / 2);
        push(mats, cd(1, 0)); push(mats, cd(0, 0)); push(mats, cd(0, 0)); push(mats, cd(1, 0));
        prog.rops.push_back(nop);
    }
}

}  // namespace qsv

namespace qsv {
dev::TileOp lower_to_lds(const Op &op, const int *li, std::vector<double> &mats, int elem_bytes) {
    double fl = 0.0;
    return lds_form(op, li, mats, elem_bytes, &fl);
}
}  // namespace qsv
