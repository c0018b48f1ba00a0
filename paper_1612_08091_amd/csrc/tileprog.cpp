// Lowering of a planned pass into the instruction list of a tile kernel.
//
// For the register-resident kernel (m = RB + 8 or RB + 9 tile bits, 2^RB
// amplitudes per thread) this decides, op by op, which tile bits live in
// registers: a 1- or 2-qubit operation needs its targets there; when it finds
// them absent a REMAP moves the tile through LDS into a layout holding the
// targets plus the bits used soonest afterwards (Belady's furthest-next-use
// rule applied to the RB register slots).  Diagonal operations run in any
// layout; passes with wider operations run on the LDS-tile kernel.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>

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

}  // namespace

uint32_t remap_offset(uint32_t l, int kept, int elem_bytes) {
    const uint32_t lowm = (1u << kept) - 1;
    const uint32_t h = ((l >> 1) & ~lowm) | (l & lowm);
    return swz_elem(h, elem_bytes) * (uint32_t)elem_bytes;
}


// ------------------------------------------------------------- real split
bool real_split(const std::vector<cd> &U, int k, std::vector<cd> &l, std::vector<double> &M,
                std::vector<cd> &rr) {
    const int d = 1 << k;
    double amax = 0.0;
    for (const cd &v : U) amax = std::max(amax, std::abs(v));
    if (!(amax > 0.0)) return false;
    // Phases travel along the entries that are clearly nonzero: breadth-first
    // over the bipartite graph of rows and columns they join.  Each phase is
    // fixed modulo pi only (M may be negative), and the representative with
    // a positive real part (or +i) is taken, so a real matrix gets phases 1.
    const double edge = 1e-6 * amax;
    auto canon = [](cd z) {
        if (z.real() < 0.0 || (z.real() == 0.0 && z.imag() < 0.0)) z = -z;
        return z;
    };
    l.assign(d, cd(1, 0));
    rr.assign(d, cd(1, 0));
    std::vector<char> lset(d, 0), rset(d, 0);
    std::vector<int> q;
    for (int r0 = 0; r0 < d; ++r0) {
        if (lset[r0]) continue;
        lset[r0] = 1;
        q.assign(1, r0);
        for (size_t h = 0; h < q.size(); ++h) {
            const int v = q[h];
            if (v < d) {
                for (int c = 0; c < d; ++c) {
                    const cd u = U[(size_t)v * d + c];
                    if (rset[c] || std::abs(u) <= edge) continue;
                    rr[c] = canon((u / std::abs(u)) * std::conj(l[v]));
                    rset[c] = 1;
                    q.push_back(d + c);
                }
            } else {
                const int c = v - d;
                for (int r = 0; r < d; ++r) {
                    const cd u = U[(size_t)r * d + c];
                    if (lset[r] || std::abs(u) <= edge) continue;
                    l[r] = canon((u / std::abs(u)) * std::conj(rr[c]));
                    lset[r] = 1;
                    q.push_back(r);
                }
            }
        }
    }
    M.assign((size_t)d * d, 0.0);
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            const cd v = U[(size_t)r * d + c] * std::conj(l[r]) * std::conj(rr[c]);
            if (std::abs(v.imag()) > 1e-14) return false;
            M[(size_t)r * d + c] = v.real();
        }
    return true;
}

namespace {

// Register-kernel layout: register slot j holds tile bit reg[j], thread-id
// bit t holds tile bit thr[t].
struct Layout {
    uint8_t reg[8] = {};
    uint8_t thr[16] = {};
};

Layout make_layout(uint32_t regmask, int m) {
    Layout L;
    int j = 0, i = 0;
    for (int b = 0; b < m; ++b) {
        if ((regmask >> b) & 1) L.reg[j++] = (uint8_t)b;
        else L.thr[i++] = (uint8_t)b;
    }
    return L;
}

// The layout after a remap to register set Sn: the register slots as
// make_layout orders them (the caller puts the kept bit back in its slot);
// thread-id bits keep their tile bits where those stay outside the
// registers, and the bits that leave the registers fill the freed slots.
// A freed wave-id slot takes the leaving bit used last (next_use), so the
// wave-id bits change as rarely as possible.
Layout next_layout(const Layout &cur, uint32_t Sn, int m, int rb, int lane_bits,
                   const int *next_use) {
    Layout nw = make_layout(Sn, m);
    const int tb = m - rb;
    uint8_t thr[16];
    bool fixed[16] = {};
    std::vector<int> leaving;
    for (int j = 0; j < rb; ++j)
        if (!((Sn >> cur.reg[j]) & 1)) leaving.push_back(cur.reg[j]);
    std::sort(leaving.begin(), leaving.end(),
              [&](int x, int y) { return next_use[x] > next_use[y]; });
    for (int t = 0; t < tb; ++t)
        if (!((Sn >> cur.thr[t]) & 1)) {
            thr[t] = cur.thr[t];
            fixed[t] = true;
        }
    size_t k = 0;
    for (int t = tb - 1; t >= lane_bits; --t)
        if (!fixed[t]) thr[t] = (uint8_t)leaving[k++];
    for (int t = 0; t < lane_bits && t < tb; ++t)
        if (!fixed[t]) thr[t] = (uint8_t)leaving[k++];
    std::memcpy(nw.thr, thr, (size_t)tb);
    return nw;
}

// A unit of the register program before lowering.
struct Item {
    int kind = dev::ROP_G1;    // ROP_G1/G2/R1/R2/DIAG
    uint32_t need = 0;         // tile bits that must be register bits
    uint64_t all = 0, mix = 0; // qubits touched / qubits whose value may change
    Op op;                     // G/R: targets, controls (G: the matrix)
    std::vector<double> rm;    // R: real matrix over op.t, row-major
    std::vector<Op> members;   // DIAG: the diagonal ops multiplied into one table
};

Op diag_op(const int *t, int k, uint64_t ctrl, const std::vector<cd> &val) {
    Op d;
    d.kind = Op::MONO;
    d.diag = true;
    d.k = k;
    for (int j = 0; j < k; ++j) d.t[j] = t[j];
    d.ctrl = ctrl;
    d.U = val;
    d.touch = 0;
    for (int r = 0; r < (1 << k); ++r) {
        d.perm[r] = (uint8_t)r;
        if (val[r] != cd(1, 0)) d.touch |= 1u << r;
    }
    return d;
}

bool all_ones(const std::vector<cd> &v) {
    for (const cd &z : v)
        if (z != cd(1, 0)) return false;
    return true;
}

// Pending image block: a table or a run of lane words, placed at the end.
struct ImgBlock {
    std::vector<unsigned char> bytes;
    uint32_t align = 16;
    int op = -1;          // index into rops
    bool table = false;   // patches rops[op].mat (else lane_off)
    bool ones = false;    // a table of ones: patches rops[op].b instead
    uint32_t off = 0;
};

void put_complex(std::vector<unsigned char> &b, const cd &v, int elem_bytes) {
    if (elem_bytes == 16) {
        double x[2] = {v.real(), v.imag()};
        const unsigned char *p = reinterpret_cast<const unsigned char *>(x);
        b.insert(b.end(), p, p + 16);
    } else {
        float x[2] = {(float)v.real(), (float)v.imag()};
        const unsigned char *p = reinterpret_cast<const unsigned char *>(x);
        b.insert(b.end(), p, p + 8);
    }
}

void put_words(std::vector<unsigned char> &b, const uint32_t *w, int n) {
    const unsigned char *p = reinterpret_cast<const unsigned char *>(w);
    b.insert(b.end(), p, p + 4 * n);
}

}  // namespace

// Lowering of one pass.  For the register kernel:
//  1. every 1- or 2-qubit op is split, when it can be, into diagonal phases
//     on either side of a real matrix (real_split); the real matrix costs
//     half the arithmetic of the complex one;
//  2. diagonal ops (the pass's own and those phases) are gathered: each may
//     move between the non-diagonal ops it commutes with, and a greedy
//     interval stabbing places them at as few points as possible, where they
//     multiply into tables of at most kRegDiagMax bits;
//  3. list scheduling orders the commuting ops to need few layout changes,
//     and Belady's furthest-next-use rule picks the register set of each
//     REMAP;
//  4. every layout-dependent offset (table indices, LDS buffer offsets,
//     per-lane words of the image) is computed here, so the kernel does no
//     layout arithmetic.
void compile_pass(const Pass &ps, int rb, std::vector<double> &mats, TileProgram &prog,
                  int elem_bytes) {
    prog = TileProgram();
    prog.tile = ps.tile;
    int li[64];
    int m = 0;
    uint8_t tpos[64];
    for (int p = 0; p < 64; ++p) {
        li[p] = -1;
        if ((ps.tile >> p) & 1) {
            tpos[m] = (uint8_t)p;
            li[p] = m++;
        }
    }
    prog.m = m;
    // store position of each tile bit (a relabeling pass moves its qubits)
    uint8_t spos[64];
    for (int b = 0; b < m; ++b) {
        spos[b] = ps.dest.empty() ? tpos[b] : ps.dest[tpos[b]];
        prog.spos[b] = spos[b];
        if (spos[b] != tpos[b]) prog.permutes = true;
    }
    // A relabeling pass stores amplitudes to addresses that other threads of
    // the workgroup load (of other waves too): all loads must be complete
    // before the first store.
    prog.store_sync = prog.permutes;
    const int tb = m - rb;
    prog.reg = rb >= 3 && rb <= 5 && (tb == 8 || (tb == 9 && rb <= 4));
    // the register kernel runs 1- and 2-qubit ops on tile qubits and diagonal ops
    for (const Op &op : ps.ops) {
        if (op.kind == Op::MONO && (op.diag || op.touch == 0)) continue;
        bool inside = true;
        for (int j = 0; j < op.k; ++j)
            if (li[op.t[j]] < 0) inside = false;
        if (!inside || op.k > 2) prog.reg = false;
    }
    auto lds_program = [&]() {
        prog.reg = false;
        prog.rops.clear();
        prog.img.clear();
        prog.flops_per_amp = 0.0;
        for (const Op &op : ps.ops) {
            if (op.kind == Op::MONO && op.touch == 0) continue;
            double fl = 0.0;
            dev::TileOp t = lds_form(op, li, mats, elem_bytes, &fl);
            prog.flops_per_amp += fl;
            if (t.kind == dev::TOP_DENSE_MFMA) prog.mfma_k = std::max(prog.mfma_k, t.k);
            prog.lops.push_back(t);
        }
    };
    if (!prog.reg) {
        lds_program();
        return;
    }
    const size_t mats_mark = mats.size();
    const uint64_t tile_mask = ps.tile;

    // ---- 1. items in queue order; diagonal pieces remember their position
    std::vector<Item> nd;                       // non-diagonal items
    struct DPiece {
        Op op;
        int pos;                                // number of nd items before it
    };
    std::vector<DPiece> dps;
    for (const Op &op : ps.ops) {
        if (op.kind == Op::MONO && op.touch == 0) continue;
        if (op.kind == Op::MONO && op.diag) {
            dps.push_back({op, (int)nd.size()});
            continue;
        }
        Item it;
        it.op = op;
        it.all = op.qubits();
        it.mix = op.mixing();
        for (int j = 0; j < op.k; ++j) it.need |= 1u << li[op.t[j]];
        const std::vector<cd> U = dense_matrix(op);
        std::vector<cd> lph, rph;
        if (real_split(U, op.k, lph, it.rm, rph)) {
            it.kind = op.k == 1 ? dev::ROP_R1 : dev::ROP_R2;
            if (!all_ones(rph)) dps.push_back({diag_op(op.t, op.k, op.ctrl, rph), (int)nd.size()});
            nd.push_back(std::move(it));
            if (!all_ones(lph)) dps.push_back({diag_op(op.t, op.k, op.ctrl, lph), (int)nd.size()});
            prog.real_ops += 1;
        } else {
            it.kind = op.k == 1 ? dev::ROP_G1 : dev::ROP_G2;
            it.rm.clear();
            nd.push_back(std::move(it));
        }
    }
    // ---- 2. the items in queue order, each diagonal piece an item of its own
    std::vector<Item> items;
    {
        const int K = (int)nd.size();
        size_t d = 0;
        items.reserve(nd.size() + dps.size());
        for (int g = 0; g <= K; ++g) {
            for (; d < dps.size() && dps[d].pos == g; ++d) {
                Item t;
                t.kind = dev::ROP_DIAG;
                t.all = dps[d].op.qubits();
                t.members.push_back(dps[d].op);
                items.push_back(std::move(t));
            }
            if (g < K) items.push_back(nd[g]);
        }
    }
    // ---- 3. list scheduling (see above), with the diagonal pieces as single
    // items (merged tables would tie the order of every op on their qubits); the first unscheduled op is always
    // ready, and the choice is among the next kWin unscheduled ops
    {
        constexpr int kWin = 256;
        const int N = (int)items.size();
        std::vector<int> npred(N, 0);
        std::vector<std::vector<int>> succ(N);
        for (int i = 0; i < N; ++i)
            for (int j = std::max(0, i - kWin); j < i; ++j)
                if (!commute_masks(items[j].mix, items[j].all, items[i].mix, items[i].all)) {
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
        std::vector<int> order;
        order.reserve(N);
        int first = 0;
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
            order.push_back(pick);
            for (int j : succ[pick])
                if (--npred[j] == 0) ready[j] = 1;
        }
        std::vector<Item> sorted;
        sorted.reserve(N);
        for (int i : order) sorted.push_back(std::move(items[i]));
        items.swap(sorted);
    }
    const std::vector<Item> scheduled = std::move(items);

    // Steps 3b-4 build the program with tables of at most `cap` qubits and
    // return the size of its LDS image.
    const int real_ops = prog.real_ops;
    auto lower = [&](int cap) -> uint32_t {
    mats.resize(mats_mark);
    prog.rops.clear();
    prog.img.clear();
    prog.remaps = prog.diag_ops = prog.diag_merged = prog.local_remaps = 0;
    prog.real_ops = real_ops;
    prog.flops_per_amp = 0.0;
    // ---- 3b. diagonal grouping by interval stabbing in the scheduled order:
    // each piece may move between the non-diagonal items it commutes with;
    // greedy stabbing (by right end) places them at as few gaps as possible
    std::vector<const Item *> nds;
    std::vector<std::pair<const Item *, int>> pcs;   // piece, nd items before it
    for (const Item &it : scheduled) {
        if (it.kind == dev::ROP_DIAG) pcs.push_back({&it, (int)nds.size()});
        else nds.push_back(&it);
    }
    const int K = (int)nds.size();
    std::vector<std::vector<int>> at_gap(K + 1);   // pieces placed before nds[g]
    {
        std::vector<int> L(pcs.size()), R(pcs.size()), order(pcs.size());
        for (size_t d = 0; d < pcs.size(); ++d) {
            const uint64_t all = pcs[d].first->all;
            int lo = 0, hi = K;
            for (int j = pcs[d].second - 1; j >= 0; --j)
                if (!commute_masks(nds[j]->mix, nds[j]->all, 0, all)) { lo = j + 1; break; }
            for (int j = pcs[d].second; j < K; ++j)
                if (!commute_masks(nds[j]->mix, nds[j]->all, 0, all)) { hi = j; break; }
            L[d] = lo;
            R[d] = hi;
            order[d] = (int)d;
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return R[x] < R[y]; });
        int stab = -1;
        for (int d : order) {
            if (L[d] > stab) stab = R[d];
            at_gap[stab].push_back(d);
        }
    }
    // pieces of one gap multiply into tables of at most `cap` qubits (first
    // fit; diagonal ops commute, so any grouping is exact)
    std::vector<Item> items;
    items.reserve(nds.size() + pcs.size());
    for (int g = 0; g <= K; ++g) {
        std::sort(at_gap[g].begin(), at_gap[g].end());
        std::vector<Item> tabs;
        for (int d : at_gap[g]) {
            const Item &pc = *pcs[d].first;
            Item *dst = nullptr;
            for (Item &t : tabs)
                if (popc(t.all | pc.all) <= cap) { dst = &t; break; }
            if (!dst) {
                tabs.emplace_back();
                dst = &tabs.back();
                dst->kind = dev::ROP_DIAG;
            } else {
                prog.diag_merged += 1;
            }
            dst->all |= pc.all;
            dst->members.insert(dst->members.end(), pc.members.begin(), pc.members.end());
        }
        for (Item &t : tabs) items.push_back(std::move(t));
        if (g < K) items.push_back(*nds[g]);
    }

    // ---- 4. lowering
    const int n_items = (int)items.size();
    const int nr = 1 << rb;
    const int lane_bits = 6;
    const int nwaves = 1 << (tb - lane_bits);
    std::vector<int> next_at((size_t)(n_items + 1) * m, 1 << 30);
    for (int i = n_items - 1; i >= 0; --i)
        for (int b = 0; b < m; ++b)
            next_at[(size_t)i * m + b] =
                ((items[i].need >> b) & 1) ? i : next_at[(size_t)(i + 1) * m + b];
    uint32_t S = 0;
    for (const Item &it : items) {
        if (__builtin_popcount(S | it.need) > rb) break;
        S |= it.need;
        if (__builtin_popcount(S) == rb) break;
    }
    for (int b = m - 1; b >= 0 && __builtin_popcount(S) < rb; --b) S |= 1u << b;
    Layout cur = make_layout(S, m);
    {
        // the wave-id bits take the thread bits whose first use is latest
        // (lane bits 0-2 keep the three lowest tile bits: contiguous loads)
        std::vector<int> cand;
        for (int t = 3; t < tb; ++t) cand.push_back(cur.thr[t]);
        std::stable_sort(cand.begin(), cand.end(),
                         [&](int x, int y) { return next_at[x] > next_at[y]; });
        const int nwb = tb - lane_bits;
        std::vector<int> wb(cand.begin(), cand.begin() + nwb), lb(cand.begin() + nwb, cand.end());
        std::sort(wb.begin(), wb.end());
        std::sort(lb.begin(), lb.end());
        for (int t = 3; t < lane_bits; ++t) cur.thr[t] = (uint8_t)lb[t - 3];
        for (int t = lane_bits; t < tb; ++t) cur.thr[t] = (uint8_t)wb[t - lane_bits];
    }
    std::memcpy(prog.reg_lbit, cur.reg, 8);
    std::memcpy(prog.thr_lbit, cur.thr, 16);
    for (int j = 0; j < rb; ++j) prog.g_reg[j] = 1ull << tpos[cur.reg[j]];
    for (int t = 0; t < tb; ++t) prog.g_thr[t] = 1ull << tpos[cur.thr[t]];
    std::vector<ImgBlock> blocks;

    // A remap that leaves the tile bits of the wave-id bits where they are
    // moves data only within each wave: it runs on the wave's own region of
    // the buffer (index over the register and lane bits), with no workgroup
    // barrier (b = 1).  Otherwise the whole workgroup exchanges through the
    // buffer; b = 2 adds a barrier before its writes when a wave-local remap
    // ran since the last workgroup barrier (another wave may still be reading
    // its region).
    bool local_since_barrier = false;
    auto emit_remap = [&](const Layout &nw, int split) {
        dev::RegOp r{};
        r.kind = dev::ROP_REMAP;
        r.a = split;
        bool local = true;
        uint32_t wmask = 0;
        for (int t = lane_bits; t < tb; ++t) {
            if (cur.thr[t] != nw.thr[t]) local = false;
            wmask |= 1u << cur.thr[t];
        }
        // Buffer address of the amplitude with local index l: a linear map
        // of its tile bits other than the kept register bit (and, wave-local,
        // the wave-id bits).  The lane bits 0..q-1 of the old layout take
        // index bits 0..q-1 (q = 4 for 16-byte, 5 for 8-byte elements: the
        // lanes a write serves together then hit distinct bank slots), and
        // each of the new layout's lane bits 0..q-1 that lies higher is
        // folded (XOR) onto the slot of an old lane bit the new layout does
        // not use, so the reads are conflict-free too.  Triangular, hence a
        // bijection onto the buffer.
        const uint32_t drop = (local ? wmask : 0u) | (1u << cur.reg[split]);
        const int q = elem_bytes == 16 ? 4 : 5;
        int pos[32];
        for (int b = 0; b < 32; ++b) pos[b] = -1;
        int np = 0;
        uint32_t A = 0, B = 0;
        for (int t = 0; t < q; ++t) {
            A |= 1u << cur.thr[t];
            B |= 1u << nw.thr[t];
        }
        for (int t = 0; t < q; ++t) pos[cur.thr[t]] = np++;
        for (int b = 0; b < m; ++b)
            if (!((drop >> b) & 1) && pos[b] < 0) pos[b] = np++;
        uint32_t fold[32] = {};
        {
            std::vector<int> from, to;
            for (int b = 0; b < m; ++b)
                if (((B >> b) & 1) && !((A >> b) & 1)) from.push_back(b);
            for (int t = 0; t < q; ++t)
                if (!((B >> cur.thr[t]) & 1)) to.push_back(pos[cur.thr[t]]);
            for (size_t k = 0; k < from.size() && k < to.size(); ++k) fold[from[k]] = 1u << to[k];
        }
        auto off = [&](uint32_t l) {
            uint32_t h = 0;
            for (int b = 0; b < m; ++b)
                if (((l >> b) & 1) && pos[b] >= 0) h ^= (1u << pos[b]) ^ fold[b];
            return h * (uint32_t)elem_bytes;
        };
        for (int i = 0; i < nr; ++i) {
            uint32_t lo = 0, ln = 0;
            for (int j = 0; j < rb; ++j)
                if ((i >> j) & 1) {
                    lo |= 1u << cur.reg[j];
                    ln |= 1u << nw.reg[j];
                }
            r.wr[i] = off(lo);
            r.rd[i] = off(ln);
        }
        uint32_t words[128];
        for (int l = 0; l < 64; ++l) {
            uint32_t w = 0, rd = 0;
            for (int t = 0; t < lane_bits; ++t)
                if ((l >> t) & 1) {
                    w ^= off(1u << cur.thr[t]);
                    rd ^= off(1u << nw.thr[t]);
                }
            words[l] = w;
            words[64 + l] = rd;
        }
        const uint32_t region = ((uint32_t)elem_bytes << (m - 1)) / (uint32_t)nwaves;
        for (int w = 0; w < nwaves; ++w) {
            uint32_t a = 0, b = 0;
            if (local) {
                a = b = (uint32_t)w * region;
            } else {
                for (int t = lane_bits; t < tb; ++t)
                    if ((w >> (t - lane_bits)) & 1) {
                        a ^= off(1u << cur.thr[t]);
                        b ^= off(1u << nw.thr[t]);
                    }
            }
            r.wwave[w] = a;
            r.rwave[w] = b;
        }
        if (local) {
            r.b = 1;
            local_since_barrier = true;
            prog.local_remaps += 1;
        } else {
            r.b = local_since_barrier ? 2 : 0;
            local_since_barrier = false;
        }
        ImgBlock blk;
        put_words(blk.bytes, words, 128);
        blk.op = (int)prog.rops.size();
        blocks.push_back(std::move(blk));
        prog.rops.push_back(r);
        prog.remaps += 1;
        cur = nw;
    };
    auto slot_of = [&](int pos) {
        const int lb = li[pos];
        for (int j = 0; j < rb; ++j)
            if (lb >= 0 && cur.reg[j] == lb) return j;
        return -1;
    };
    auto thr_of = [&](int pos) {
        const int lb = li[pos];
        for (int t = 0; t < tb; ++t)
            if (lb >= 0 && cur.thr[t] == lb) return t;
        return -1;
    };

    for (int i = 0; i < n_items; ++i) {
        Item &it = items[i];
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
            // the two-phase remap needs one tile bit that stays in its register
            // slot: keep the old register bit used soonest if none survived
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
            int split = -1;
            for (int j = 0; j < rb; ++j)
                if (((Sn >> cur.reg[j]) & 1) &&
                    (split < 0 || next_use[cur.reg[j]] < next_use[cur.reg[split]]))
                    split = j;
            Layout nw = next_layout(cur, Sn, m, rb, lane_bits, next_use);
            for (int j = 0; j < rb; ++j)
                if (nw.reg[j] == cur.reg[split]) std::swap(nw.reg[j], nw.reg[split]);
            emit_remap(nw, split);
            S = Sn;
        }
        dev::RegOp r{};
        r.kind = it.kind;
        if (it.kind == dev::ROP_DIAG) {
            // table bits: every qubit of the members except the controls that
            // all of them share and that lie outside the tile
            uint64_t common = ~0ull;
            for (const Op &o : it.members) common &= o.ctrl;
            const uint64_t octrl = common & ~tile_mask;
            const uint64_t tq_mask = it.all & ~octrl;
            // table bit order: the qubits on lane bits first, by lane bit, so
            // that the 16 lanes a ds_read_b128 serves together (lane bits 0-3)
            // read distinct 16-byte slots of one 256-byte bank row, or the
            // same slot (a broadcast): no bank conflicts
            int tq[dev::kRegDiagMax], kt = 0;
            for (int t = 0; t < lane_bits; ++t)
                for (int p = 0; p < 64; ++p)
                    if (((tq_mask >> p) & 1) && li[p] >= 0 && slot_of(p) < 0 && thr_of(p) == t)
                        tq[kt++] = p;
            for (int p = 0; p < 64; ++p) {
                if (!((tq_mask >> p) & 1)) continue;
                const int t = li[p] >= 0 && slot_of(p) < 0 ? thr_of(p) : -1;
                if (t < 0 || t >= lane_bits) tq[kt++] = p;
            }
            r.octrl = octrl;
            const uint32_t eb = (uint32_t)elem_bytes;
            for (int j = 0; j < kt; ++j) {
                const uint32_t wgt = eb << j;
                if (li[tq[j]] < 0) {
                    r.gt[r.a] = (uint32_t)tq[j];
                    r.gtb[r.a] = wgt;
                    r.a += 1;
                    continue;
                }
                const int sj = slot_of(tq[j]);
                if (sj >= 0) {
                    for (int x = 0; x < nr; ++x)
                        if ((x >> sj) & 1) r.wr[x] |= wgt;
                } else {
                    const int t = thr_of(tq[j]);
                    if (t >= lane_bits)
                        for (int w = 0; w < nwaves; ++w)
                            if ((w >> (t - lane_bits)) & 1) r.wwave[w] |= wgt;
                }
            }
            // lane thread-id bit t that is table bit j: bit t of lane_ok set,
            // rd[t] = the bit's place in the byte offset (j + log2 eb)
            r.lane_ok = 0;
            for (int j = 0; j < kt; ++j) {
                const int t = li[tq[j]] >= 0 && slot_of(tq[j]) < 0 ? thr_of(tq[j]) : -1;
                if (t >= 0 && t < lane_bits) {
                    r.lane_ok |= 1ull << t;
                    r.rd[t] = (uint32_t)(j + __builtin_ctz(eb));
                }
            }
            ImgBlock tab;
            int changed = 0;
            for (uint32_t row = 0; row < (1u << kt); ++row) {
                uint64_t bits = octrl;
                for (int j = 0; j < kt; ++j)
                    if ((row >> j) & 1) bits |= 1ull << tq[j];
                cd v(1, 0);
                for (const Op &o : it.members) {
                    if ((bits & o.ctrl) != o.ctrl) continue;
                    uint32_t rix = 0;
                    for (int j = 0; j < o.k; ++j)
                        if ((bits >> o.t[j]) & 1) rix |= 1u << j;
                    v *= o.U[rix];
                }
                if (v != cd(1, 0)) ++changed;
                put_complex(tab.bytes, v, elem_bytes);
            }
            tab.align = std::max<uint32_t>(16u, eb << kt);
            tab.op = (int)prog.rops.size();
            tab.table = true;
            if (octrl) {
                // tiles that fail the controls outside the tile read ones
                ImgBlock ones;
                for (uint32_t row = 0; row < (1u << kt); ++row) put_complex(ones.bytes, cd(1, 0), elem_bytes);
                ones.align = tab.align;
                ones.op = tab.op;
                ones.table = true;
                ones.ones = true;
                blocks.push_back(std::move(ones));
            }
            blocks.push_back(std::move(tab));
            prog.diag_ops += 1;
            prog.flops_per_amp += 6.0;
            (void)changed;
        } else {
            const Op &op = it.op;
            const bool two = op.k == 2;
            const int j0 = slot_of(op.t[0]), j1 = two ? slot_of(op.t[1]) : -1;
            const bool swap01 = two && j1 < j0;
            r.a = swap01 ? j1 : j0;
            r.b = two ? (swap01 ? j0 : j1) : 0;
            // controls: register bits, thread-id bits (lane and wave masks),
            // and bits outside the tile
            r.lane_ok = ~0ull;
            r.wave_ok = ~0u;
            for (int p = 0; p < 64; ++p) {
                if (!((op.ctrl >> p) & 1)) continue;
                if (li[p] < 0) {
                    r.octrl |= 1ull << p;
                    continue;
                }
                const int sj = slot_of(p);
                if (sj >= 0) {
                    r.creg |= 1u << sj;
                    continue;
                }
                const int t = thr_of(p);
                if (t < lane_bits) {
                    uint64_t lm = 0;
                    for (int l = 0; l < 64; ++l)
                        if ((l >> t) & 1) lm |= 1ull << l;
                    r.lane_ok &= lm;
                } else {
                    uint32_t wm = 0;
                    for (int w = 0; w < nwaves; ++w)
                        if ((w >> (t - lane_bits)) & 1) wm |= 1u << w;
                    r.wave_ok &= wm;
                }
            }
            auto sw = [](int x) { return ((x & 1) << 1) | ((x >> 1) & 1); };
            const int D = 1 << op.k;
            const double frac = 1.0 / (double)(1ull << popc(op.ctrl));
            int e = 0;
            if (it.kind == dev::ROP_R1 || it.kind == dev::ROP_R2) {
                for (int row = 0; row < D; ++row)
                    for (int col = 0; col < D; ++col)
                        r.md[e++] = swap01 ? it.rm[(size_t)sw(row) * D + sw(col)]
                                           : it.rm[(size_t)row * D + col];
                prog.flops_per_amp += frac * (two ? 14.0 : 6.0);
            } else {
                const std::vector<cd> U = dense_matrix(op);
                for (int row = 0; row < D; ++row)
                    for (int col = 0; col < D; ++col) {
                        const cd v = swap01 ? U[(size_t)sw(row) * D + sw(col)] : U[(size_t)row * D + col];
                        r.md[e++] = v.real();
                        r.md[e++] = v.imag();
                    }
                prog.flops_per_amp += frac * (two ? 30.0 : 14.0);
            }
            for (int x = 0; x < 32; ++x) r.mf[x] = (float)r.md[x];
        }
        prog.rops.push_back(r);
    }
    // Stores leave from the final layout.  With some of the three lowest tile
    // bits in registers and the first two thread bits far up the index, each
    // store instruction writes 16-byte pieces of many separate 128-byte
    // lines, and the memory system writes them out more than once (measured:
    // 2.5 x the state for one pass of the 30-qubit brick circuit).  A final
    // remap to a layout without those bits in registers costs less.
    if (prog.permutes) {
        // A relabeling pass stores to other positions: the tile bits of the
        // three lowest store positions must be lane bits (each store
        // instruction then writes whole 128-byte lines).
        int ord[32];
        for (int b = 0; b < m; ++b) ord[b] = b;
        std::sort(ord, ord + m, [&](int x, int y) { return spos[x] < spos[y]; });
        const uint32_t low3 = (1u << ord[0]) | (1u << ord[1]) | (1u << ord[2]);
        bool lanes_ok = true;
        for (int c = 0; c < 3; ++c) {
            bool in_lane = false;
            for (int t = 0; t < lane_bits && t < tb; ++t)
                if (cur.thr[t] == ord[c]) in_lane = true;
            lanes_ok = lanes_ok && in_lane;
        }
        if (!lanes_ok) {
            uint32_t Sn = S & ~low3;
            for (int k = m - 1; k >= 0 && __builtin_popcount(Sn) < rb; --k)
                if (!((low3 >> ord[k]) & 1)) Sn |= 1u << ord[k];
            int split = -1;
            for (int j = 0; j < rb && split < 0; ++j)
                if ((Sn >> cur.reg[j]) & 1) split = j;
            if (split >= 0 && __builtin_popcount(Sn) == rb) {
                Layout nw;
                std::vector<int> regs, th;
                for (int b = 0; b < m; ++b)
                    if (((Sn >> b) & 1) && b != cur.reg[split]) regs.push_back(b);
                for (int j = 0, k = 0; j < rb; ++j)
                    nw.reg[j] = (uint8_t)(j == split ? cur.reg[split] : regs[k++]);
                for (int c = 0; c < 3; ++c) th.push_back(ord[c]);
                for (int b = 0; b < m; ++b)
                    if (!((Sn >> b) & 1) && !((low3 >> b) & 1)) th.push_back(b);
                for (int t = 0; t < tb; ++t) nw.thr[t] = (uint8_t)th[t];
                emit_remap(nw, split);
                S = Sn;
            }
        }
    } else if (S & 0x7u) {
        if (tb >= 2 && (tpos[cur.thr[0]] > 5 || tpos[cur.thr[1]] > 6)) {
            uint32_t Sn = S & ~0x7u;
            for (int b = m - 1; b >= 3 && __builtin_popcount(Sn) < rb; --b) Sn |= 1u << b;
            int split = -1;
            for (int j = 0; j < rb && split < 0; ++j)
                if ((Sn >> cur.reg[j]) & 1) split = j;
            if (split >= 0 && __builtin_popcount(Sn) == rb) {
                Layout nw = make_layout(Sn, m);
                for (int j = 0; j < rb; ++j)
                    if (nw.reg[j] == cur.reg[split]) std::swap(nw.reg[j], nw.reg[split]);
                emit_remap(nw, split);
                S = Sn;
            }
        }
    }
    // The program runs once per tile with no barrier between tiles: a
    // wave-local remap after the last workgroup remap is followed, in the
    // next tile, by the first workgroup remap, which must then wait too.
    if (local_since_barrier)
        for (dev::RegOp &r : prog.rops)
            if (r.kind == dev::ROP_REMAP && r.b != 1) {
                r.b = 2;
                break;
            }
    for (int j = 0; j < rb; ++j) prog.g_reg_f[j] = 1ull << spos[cur.reg[j]];
    for (int t = 0; t < tb; ++t) prog.g_thr_f[t] = 1ull << spos[cur.thr[t]];
    // the kernel runs ops in pairs: pad with an identity real 1-qubit op
    if (prog.rops.size() & 1) {
        dev::RegOp pad{};
        pad.kind = dev::ROP_R1;
        pad.lane_ok = ~0ull;
        pad.wave_ok = ~0u;
        pad.md[0] = pad.md[3] = 1.0;
        pad.mf[0] = pad.mf[3] = 1.0f;
        prog.rops.push_back(pad);
    }
    // LDS image: tables first, largest first (each then sits at a multiple of
    // its own size), then the lane words
    std::vector<int> ord(blocks.size());
    for (size_t b = 0; b < blocks.size(); ++b) ord[b] = (int)b;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
        if (blocks[x].table != blocks[y].table) return blocks[x].table;
        return blocks[x].align > blocks[y].align;
    });
    uint32_t off = 0;
    for (int b : ord) {
        ImgBlock &blk = blocks[b];
        off = (off + blk.align - 1) & ~(blk.align - 1);
        blk.off = off;
        off += (uint32_t)blk.bytes.size();
    }
    off = (off + 15u) & ~15u;
    prog.img.assign(off, 0);
    for (const ImgBlock &blk : blocks) {
        std::memcpy(prog.img.data() + blk.off, blk.bytes.data(), blk.bytes.size());
        if (blk.ones) prog.rops[blk.op].b = (int32_t)blk.off;
        else if (blk.table) prog.rops[blk.op].mat = blk.off;
        else prog.rops[blk.op].lane_off = blk.off;
    }
    return off;
    };
    // The widest tables that keep the image within kRegImageSoft (three
    // workgroups per compute unit with a 12-bit complex128 tile); narrower
    // tables mean more table ops but a smaller image.  An image past
    // kRegImageMax sends the pass to the LDS-tile kernel.
    static const int caps[] = {dev::kRegDiagMax, 6, 4, 3, 2};
    uint32_t img = 0;
    for (int cap : caps) {
        img = lower(cap);
        if (img <= dev::kRegImageSoft) break;
    }
    if (img > dev::kRegImageMax) {
        mats.resize(mats_mark);
        prog.rops.clear();
        prog.img.clear();
        prog.real_ops = prog.diag_ops = prog.remaps = prog.diag_merged = 0;
        lds_program();
    }
}

// ------------------------------------------------------------- host model
std::string emulate_reg_pass(const TileProgram &prog, int rb, const std::vector<double> &mats,
                             int elem_bytes, int n, std::vector<cd> &state) {
    if (!prog.reg) return "not a register program";
    const int m = prog.m, tb = m - rb, nt = 1 << tb, nr = 1 << rb;
    if (n < m) return "state smaller than the tile";
    uint8_t tpos[64];
    int c = 0;
    for (int p = 0; p < 64; ++p)
        if ((prog.tile >> p) & 1) tpos[c++] = (uint8_t)p;
    if (c != m) return "tile mask and m disagree";
    const uint32_t half = (uint32_t)elem_bytes << (m - 1);
    const size_t img = prog.img.size();
    auto rd_u32 = [&](uint32_t off, uint32_t *out) -> bool {
        if (off % 4 || (size_t)off + 4 > img) return false;
        std::memcpy(out, prog.img.data() + off, 4);
        return true;
    };
    auto rd_cplx = [&](uint32_t off, cd *out) -> bool {
        if (off % (uint32_t)elem_bytes || (size_t)off + elem_bytes > img) return false;
        if (elem_bytes == 16) {
            double x[2];
            std::memcpy(x, prog.img.data() + off, 16);
            *out = cd(x[0], x[1]);
        } else {
            float x[2];
            std::memcpy(x, prog.img.data() + off, 8);
            *out = cd(x[0], x[1]);
        }
        return true;
    };
    auto gidx = [&](const uint64_t *g_reg, const uint64_t *g_thr, int t, int i) {
        uint64_t x = 0;
        for (int j = 0; j < rb; ++j)
            if ((i >> j) & 1) x |= g_reg[j];
        for (int s = 0; s < tb; ++s)
            if ((t >> s) & 1) x |= g_thr[s];
        return x;
    };
    const uint64_t n_tiles = 1ull << (n - m);
    std::vector<cd> amp((size_t)nt * nr);
    std::vector<cd> buf(half / elem_bytes);
    std::vector<char> full(half / elem_bytes);
    std::vector<char> seen((size_t)1 << m);
    std::vector<int> loaded_by((size_t)1 << m, -1);
    bool wg_synced = prog.store_sync, wave_synced = false;
    for (const dev::RegOp &op : prog.rops)
        if (op.kind == dev::ROP_REMAP) {
            if (op.b == 1) wave_synced = true;
            else wg_synced = true;
        }
    char msg[256];
    for (uint64_t tile = 0; tile < n_tiles; ++tile) {
        uint64_t base = tile;
        for (int i = 0; i < m; ++i) {
            const uint64_t lowm = (1ull << tpos[i]) - 1;
            base = ((base & ~lowm) << 1) | (base & lowm);
        }
        for (int t = 0; t < nt; ++t)
            for (int i = 0; i < nr; ++i) {
                const uint64_t x = gidx(prog.g_reg, prog.g_thr, t, i);
                if (x & ~prog.tile) return "load index outside the tile";
                uint64_t lx = 0;
                for (int b = 0; b < m; ++b)
                    if ((x >> tpos[b]) & 1) lx |= 1ull << b;
                loaded_by[lx] = t;
                amp[(size_t)t * nr + i] = state[base | x];
            }
        for (size_t oi = 0; oi < prog.rops.size(); ++oi) {
            const dev::RegOp &op = prog.rops[oi];
            if (op.kind == dev::ROP_REMAP) {
                const int J = op.a;
                // a wave-local remap (b = 1) must keep every wave inside its
                // own region of the buffer: no barrier orders it against the
                // other waves
                const uint32_t region = half >> (tb - 6);
                auto in_region = [&](int t, uint32_t a) {
                    return op.b != 1 || (a / region == (uint32_t)(t >> 6));
                };
                for (int p = 0; p < 2; ++p) {
                    std::fill(full.begin(), full.end(), 0);
                    for (int t = 0; t < nt; ++t) {
                        uint32_t lw;
                        if (!rd_u32(op.lane_off + 4 * (t & 63), &lw)) return "remap lane word out of the image";
                        const uint32_t wt = lw ^ op.wwave[t >> 6];
                        for (int i = 0; i < nr; ++i) {
                            if (((i >> J) & 1) != p) continue;
                            const uint32_t a = wt ^ op.wr[i];
                            if (a % elem_bytes || a >= half) {
                                std::snprintf(msg, sizeof msg, "op %zu: remap write at %u (buffer %u)", oi, a, half);
                                return msg;
                            }
                            if (!in_region(t, a)) return "wave-local remap writes outside its wave's region";
                            if (full[a / elem_bytes]) return "remap writes one slot twice";
                            full[a / elem_bytes] = 1;
                            buf[a / elem_bytes] = amp[(size_t)t * nr + i];
                        }
                    }
                    for (int t = 0; t < nt; ++t) {
                        uint32_t lw;
                        if (!rd_u32(op.lane_off + 256 + 4 * (t & 63), &lw)) return "remap lane word out of the image";
                        const uint32_t rt = lw ^ op.rwave[t >> 6];
                        for (int i = 0; i < nr; ++i) {
                            if (((i >> J) & 1) != p) continue;
                            const uint32_t a = rt ^ op.rd[i];
                            if (a % elem_bytes || a >= half) return "remap read outside the buffer";
                            if (!in_region(t, a)) return "wave-local remap reads outside its wave's region";
                            if (full[a / elem_bytes] != 1) return "remap reads a slot not written (or twice)";
                            full[a / elem_bytes] = 2;
                            amp[(size_t)t * nr + i] = buf[a / elem_bytes];
                        }
                    }
                }
                continue;
            }
            if (op.kind == dev::ROP_DIAG) {
                uint32_t s_idx = (uint32_t)op.mat;
                if ((base & op.octrl) != op.octrl) s_idx = (uint32_t)op.b;
                for (int q = 0; q < op.a; ++q)
                    if ((base >> op.gt[q]) & 1) s_idx ^= op.gtb[q];
                for (int t = 0; t < nt; ++t) {
                    uint32_t lw = 0;
                    for (int b = 0; b < 6; ++b)
                        if ((op.lane_ok >> b) & 1) lw |= (uint32_t)(((t & 63) >> b) & 1) << op.rd[b];
                    const uint32_t v_idx = lw ^ s_idx ^ op.wwave[t >> 6];
                    for (int i = 0; i < nr; ++i) {
                        cd f;
                        if (!rd_cplx(v_idx ^ op.wr[i], &f)) return "diag table read out of the image";
                        amp[(size_t)t * nr + i] *= f;
                    }
                }
                continue;
            }
            const bool two = op.kind == dev::ROP_G2 || op.kind == dev::ROP_R2;
            const bool real = op.kind == dev::ROP_R1 || op.kind == dev::ROP_R2;
            const int D = two ? 4 : 2;
            auto mval = [&](int x) { return elem_bytes == 16 ? op.md[x] : (double)op.mf[x]; };
            const int off[4] = {0, 1 << op.a, two ? (1 << op.b) : 0,
                                two ? ((1 << op.a) | (1 << op.b)) : 0};
            const int tmask = two ? ((1 << op.a) | (1 << op.b)) : (1 << op.a);
            if ((base & op.octrl) != op.octrl) continue;
            for (int t = 0; t < nt; ++t) {
                if (!((op.wave_ok >> (t >> 6)) & 1)) continue;
                if (!((op.lane_ok >> (t & 63)) & 1)) continue;
                for (int i = 0; i < nr; ++i) {
                    if (i & tmask) continue;
                    if ((i & (int)op.creg) != (int)op.creg) continue;
                    cd x[4], y[4];
                    for (int cc = 0; cc < D; ++cc) x[cc] = amp[(size_t)t * nr + (i | off[cc])];
                    for (int rr = 0; rr < D; ++rr) {
                        y[rr] = 0;
                        for (int cc = 0; cc < D; ++cc) {
                            const size_t e = (size_t)rr * D + cc;
                            const cd u = real ? cd(mval((int)e), 0.0)
                                              : cd(mval(2 * (int)e), mval(2 * (int)e + 1));
                            y[rr] += u * x[cc];
                        }
                    }
                    for (int rr = 0; rr < D; ++rr) amp[(size_t)t * nr + (i | off[rr])] = y[rr];
                }
            }
        }
        std::fill(seen.begin(), seen.end(), 0);
        for (int t = 0; t < nt; ++t)
            for (int i = 0; i < nr; ++i) {
                const uint64_t x = gidx(prog.g_reg_f, prog.g_thr_f, t, i);
                if (x & ~prog.tile) return "store index outside the tile";
                uint64_t lx = 0;
                for (int b = 0; b < m; ++b)
                    if ((x >> tpos[b]) & 1) lx |= 1ull << b;
                if (seen[lx]) return "store writes one amplitude twice";
                seen[lx] = 1;
                // without a workgroup barrier after the loads (a workgroup
                // remap, or the store barrier) a thread may store only what
                // its own wave loaded, and without a wave-local remap only
                // what it loaded itself: the loads of others may be pending
                const int owner = loaded_by[lx];
                if (!wg_synced && (owner >> 6) != (t >> 6))
                    return "store to an amplitude another wave loads, with no barrier between";
                if (!wg_synced && !wave_synced && owner != t)
                    return "store to an amplitude another lane loads, with no exchange between";
                state[base | x] = amp[(size_t)t * nr + i];
            }
    }
    return "";
}

}  // namespace qsv

namespace qsv {
dev::TileOp lower_to_lds(const Op &op, const int *li, std::vector<double> &mats, int elem_bytes) {
    double fl = 0.0;
    return lds_form(op, li, mats, elem_bytes, &fl);
}
}  // namespace qsv
