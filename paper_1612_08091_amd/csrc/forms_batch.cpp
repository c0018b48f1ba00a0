// Batched form: many small circuits, each with its own Pauli sum, evaluated
// by launches that are captured once in a HIP graph and replayed.
//
// At creation every circuit is canonicalised, fused and planned into LDS-tile
// passes for a tile of min(n, mb) bits.  Circuits whose state fits in LDS
// (n <= mb) run in one persistent launch, ordered by decreasing estimated
// cost (longest-processing-time first) so that its workgroups finish
// together.  Larger ones run pass-major: one launch per pass index over the
// tiles of all of them (circuits of at least 13 qubits on the register-tile
// kernel, planned and lowered as a single state is), then their Pauli sums
// in chunks.  The tile bits mb and the fusion width are
// picked by timing candidate plans on the device (autotune) and remembered in
// a JSON cache keyed by device, dtype and the circuit-size histogram.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/qsv.h"
#include "device.hpp"
#include "qsv_internal.hpp"
#include "tileprog.hpp"

using qsv::cd;
using qsv::Gate;
using qsv::Op;
using qsv::Pass;

namespace {
qsv_status berr(qsv_status st, const std::string &m) {
    qsv::set_last_error(m);   // reported by qsv_last_error(NULL)
    return st;
}
}  // namespace

struct qsv_batch {
    int count = 0;
    int dtype = QSV_C64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool use_graph = true;
    // parsed circuits
    std::vector<int> nq;
    std::vector<std::vector<Op>> ops;
    std::vector<std::vector<qsv::dev::BatchTerm>> terms;
    // device plan
    void *d_buf = nullptr;
    void *d_scratch = nullptr;
    size_t scratch_bytes = 0;
    // pass-major circuits: their states, and the launches' segment ranges
    // and item counts (host copies that the launches read)
    bool big_per_wg = false;
    void *d_states = nullptr;
    size_t states_bytes = 0;
    std::vector<int32_t> h_seg_begin;
    std::vector<uint64_t> h_items;
    // register-tile programs of the circuits of at least 13 qubits (planned
    // once per circuit, on first use), and the register launches' host arrays
    struct RegPlan {
        bool done = false, ok = false;
        std::vector<qsv::TileProgram> progs;
    };
    std::vector<RegPlan> regplan;
    std::vector<int32_t> h_reg_seg_begin;
    std::vector<uint64_t> h_reg_items;
    std::vector<int32_t> h_reg_dg;
    qsv::dev::BatchLaunch L{};
    int mb = 0, kfuse = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double last_ms = 0.0;
};

namespace {

void rot(int op, double th, std::vector<cd> &U) {
    const double c = std::cos(th / 2), s = std::sin(th / 2);
    if (op == QSV_OP_RX) U = {cd(c, 0), cd(0, -s), cd(0, -s), cd(c, 0)};
    else if (op == QSV_OP_RY) U = {cd(c, 0), cd(-s, 0), cd(s, 0), cd(c, 0)};
    else U = {std::polar(1.0, -th / 2), cd(0, 0), cd(0, 0), std::polar(1.0, th / 2)};
}

qsv_status parse(const qsv_circuit &c, const qsv_pauli_sum &h, int idx, std::vector<Op> &ops,
                 std::vector<qsv::dev::BatchTerm> &terms) {
    const std::string who = "circuit " + std::to_string(idx) + ": ";
    if (c.n_qubits < 1 || c.n_qubits > 30) return berr(QSV_EINVAL, who + "n_qubits must be 1..30");
    if (c.n_gates < 0 || (c.n_gates > 0 && (!c.op || !c.k || !c.c || !c.qubits)))
        return berr(QSV_EINVAL, who + "bad gate arrays");
    for (int g = 0; g < c.n_gates; ++g) {
        const int k = c.k[g], nc = c.c[g];
        if (k < 1 || nc < 0 || k + nc > 2 || k + nc > c.n_qubits)
            return berr(QSV_EINVAL, who + "batched gates act on at most 2 qubits");
        Gate gt;
        gt.k = k;
        uint64_t seen = 0;
        for (int j = 0; j < k + nc; ++j) {
            const int q = c.qubits[8 * g + j];
            if (q < 0 || q >= c.n_qubits || ((seen >> q) & 1))
                return berr(QSV_EINVAL, who + "bad or repeated qubit");
            seen |= 1ull << q;
            if (j < k) gt.t[j] = q;
            else gt.ctrl |= 1ull << q;
        }
        const int op = c.op[g];
        if (op == QSV_OP_MATRIX) {
            if (!c.matrices || !c.mat_off) return berr(QSV_EINVAL, who + "missing matrices");
            const int D = 1 << k;
            const double *m = c.matrices + 2 * c.mat_off[g];
            gt.U.resize((size_t)D * D);
            for (int e = 0; e < D * D; ++e) {
                if (!std::isfinite(m[2 * e]) || !std::isfinite(m[2 * e + 1]))
                    return berr(QSV_EINVAL, who + "non-finite matrix entry");
                gt.U[e] = cd(m[2 * e], m[2 * e + 1]);
            }
        } else if (op >= QSV_OP_RX && op <= QSV_OP_RZ) {
            const int p = c.param ? c.param[g] : -1;
            if (k != 1 || p < 0 || p >= c.n_params || !c.params || !std::isfinite(c.params[p]))
                return berr(QSV_EINVAL, who + "bad rotation gate");
            rot(op, c.params[p], gt.U);
        } else {
            return berr(QSV_EINVAL, who + "unknown gate op");
        }
        Op o;
        if (qsv::canonicalize(gt, o)) ops.push_back(std::move(o));
    }
    if (h.n_terms < 0 || (h.n_terms > 0 && (!h.xmask || !h.zmask || !h.coeff)))
        return berr(QSV_EINVAL, who + "bad Pauli sum");
    const uint64_t full = (1ull << c.n_qubits) - 1;
    for (int t = 0; t < h.n_terms; ++t) {
        if (((h.xmask[t] | h.zmask[t]) & ~full) || !std::isfinite(h.coeff[t]))
            return berr(QSV_EINVAL, who + "Pauli term outside the circuit");
        qsv::dev::BatchTerm bt{};
        bt.x = h.xmask[t];
        bt.z = h.zmask[t];
        bt.c = h.coeff[t];
        bt.ny = qsv::popc(bt.x & bt.z);
        terms.push_back(bt);
    }
    return QSV_OK;
}

void free_plan(qsv_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (b->d_buf) (void)hipFree(b->d_buf);
    b->d_buf = nullptr;
}

// The register-tile plan of circuit i: the single-state path's planning (12-bit
// tiles, fusion to 2 qubits, relabeling) and lowering; ok = false when a pass
// does not lower to the register kernel.
constexpr int kRegMinQubits = 13;
const qsv_batch::RegPlan &reg_plan(qsv_batch *b, int i) {
    qsv_batch::RegPlan &rp = b->regplan[i];
    if (rp.done) return rp;
    rp.done = true;
    const int n = b->nq[i];
    const int elem = b->dtype == QSV_C128 ? 16 : 8;
    std::vector<Pass> ps = qsv::plan_tiled(b->ops[i], n, 12, 2, elem == 16 ? 17 : 18, true);
    std::vector<double> mats;
    for (const Pass &p : ps) {
        qsv::TileProgram pg;
        qsv::compile_pass(p, 4, mats, pg, elem);
        if (!pg.reg || pg.m != 12 || (pg.rops.size() & 1)) {
            rp.progs.clear();
            return rp;
        }
        if (pg.rops.empty() && !pg.permutes) continue;
        rp.progs.push_back(std::move(pg));
    }
    rp.ok = true;
    return rp;
}

qsv::dev::TileArgs reg_args(const qsv::TileProgram &pg, int n, int64_t img_off) {
    qsv::dev::TileArgs ta{};
    ta.m = pg.m;
    ta.nq = n;
    ta.tile_pos_n = pg.m;
    int c = 0;
    for (int p = 0; p < 64; ++p)
        if ((pg.tile >> p) & 1) ta.tpos[c++] = (uint32_t)p;
    ta.n_tiles = 1ull << (n - pg.m);
    std::memcpy(ta.g_reg, pg.g_reg, sizeof(ta.g_reg));
    std::memcpy(ta.g_thr, pg.g_thr, sizeof(ta.g_thr));
    std::memcpy(ta.g_reg_f, pg.g_reg_f, sizeof(ta.g_reg_f));
    std::memcpy(ta.g_thr_f, pg.g_thr_f, sizeof(ta.g_thr_f));
    ta.img_bytes = (uint32_t)pg.img.size();
    ta.store_sync = 1;
    ta.img_off = img_off;
    ta.rb = 4;
    ta.n_ops = (int32_t)pg.rops.size();
    ta.no_diag = 1;
    for (const qsv::dev::RegOp &r : pg.rops)
        if (r.kind == qsv::dev::ROP_DIAG) ta.no_diag = 0;
    for (int b2 = 0; b2 < pg.m; ++b2) ta.spos[b2] = pg.spos[b2];
    return ta;
}

template <typename X>
size_t put(std::vector<unsigned char> &host, const std::vector<X> &v) {
    const size_t off = (host.size() + 255) & ~size_t(255);
    host.resize(off + v.size() * sizeof(X) + 8);
    if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(X));
    return off;
}

// Plan all circuits for tile bits mb and fusion width kf, upload, fill b->L.
qsv_status build_plan(qsv_batch *b, int mb, int kf) {
    (void)hipStreamSynchronize(b->stream);
    free_plan(b);
    std::vector<qsv::dev::BatchCircuit> circ(b->count);
    std::vector<qsv::dev::BatchPass> passes;
    std::vector<qsv::dev::TileOp> tops;
    std::vector<qsv::dev::BatchTerm> terms;
    std::vector<double> mats;
    std::vector<double> cost(b->count);
    int max_big = 0;
    int mfma_k = 0;
    for (int i = 0; i < b->count; ++i) {
        const int n = b->nq[i];
        const int m = std::min(n, mb);
        std::vector<Pass> ps = qsv::plan_passes(b->ops[i], n, m, std::min(3, m - 1), kf);
        if (ps.empty() && n > mb) {
            // a state in global memory is written by its first pass
            Pass p0;
            p0.tile = (1ull << m) - 1;
            ps.push_back(p0);
        }
        qsv::dev::BatchCircuit &bc = circ[i];
        bc.n = n;
        bc.pass_begin = (int)passes.size();
        bc.pass_count = (int)ps.size();
        bc.term_begin = (int)terms.size();
        bc.term_count = (int)b->terms[i].size();
        bc.out_index = i;
        double nops = 0;
        for (const Pass &p : ps) {
            qsv::dev::BatchPass bp{};
            int li[64];
            int mm = 0;
            for (int q = 0; q < 64; ++q) {
                li[q] = -1;
                if ((p.tile >> q) & 1) {
                    li[q] = mm;
                    bp.tpos[mm++] = (uint32_t)q;
                }
            }
            bp.m = mm;
            bp.op_begin = (int)tops.size();
            for (const Op &op : p.ops) {
                if (op.kind == Op::MONO && op.touch == 0) continue;
                tops.push_back(qsv::lower_to_lds(op, li, mats, b->dtype == QSV_C128 ? 16 : 8));
                if (tops.back().kind == qsv::dev::TOP_DENSE_MFMA)
                    mfma_k = std::max(mfma_k, tops.back().k);
            }
            bp.op_count = (int)tops.size() - bp.op_begin;
            nops += bp.op_count;
            passes.push_back(bp);
        }
        terms.insert(terms.end(), b->terms[i].begin(), b->terms[i].end());
        const double dim = (double)(1ull << n);
        cost[i] = dim * (nops + 2.0 * bc.term_count + (n > mb ? 4.0 * ps.size() : 0.0));
        if (n > mb) max_big = std::max(max_big, n);
    }
    // Circuits above the LDS limit run pass-major (one launch per pass index
    // over all their tiles) when their states fit in half the free device
    // memory; otherwise, or on request, each runs on one workgroup of the
    // persistent launch in a slot of its own.
    const size_t elem = b->dtype == QSV_C128 ? 16 : 8;
    std::vector<int> big;
    uint64_t big_amps = 0;
    for (int i = 0; i < b->count; ++i)
        if (b->nq[i] > mb) {
            big.push_back(i);
            big_amps += 1ull << b->nq[i];
        }
    bool pm = !big.empty() && !b->big_per_wg;
    if (pm) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess || (double)big_amps * elem > 0.5 * (double)fr)
            pm = false;
    }
    if (pm) max_big = 0;
    std::vector<qsv::dev::BatchSeg> segs;
    b->h_seg_begin.clear();
    b->h_items.clear();
    int n_pass_launches = 0;
    // Pauli chunk per work item, held in LDS: 32 KiB
    const int kChunkLog = b->dtype == QSV_C128 ? 11 : 12;
    // register-path circuits (at least 13 qubits, every pass lowered to the
    // register kernel) and LDS-path ones; states: LDS-path first, then the
    // register-path ones in one range (set to |0...0> by one fill)
    std::vector<int> big_lds, big_reg;
    std::vector<qsv::dev::TileArgs> tas;
    std::vector<qsv::dev::RegOp> rops;
    std::vector<unsigned char> imgs;
    std::vector<qsv::dev::RegSeg> rsegs;
    std::vector<uint64_t> reg_starts;
    uint32_t img_max = 0;
    uint64_t reg_state_off = 0, reg_amps = 0;
    b->h_reg_seg_begin.clear();
    b->h_reg_items.clear();
    b->h_reg_dg.clear();
    if (pm) {
        for (int i : big) {
            if (b->nq[i] >= kRegMinQubits && reg_plan(b, i).ok) big_reg.push_back(i);
            else big_lds.push_back(i);
        }
        std::vector<uint64_t> state_off(b->count, 0);
        uint64_t off = 0;
        for (int i : big_lds) {
            state_off[i] = off;
            off += 1ull << b->nq[i];
        }
        reg_state_off = off;
        for (int i : big_reg) {
            state_off[i] = off;
            reg_starts.push_back(off);
            off += 1ull << b->nq[i];
        }
        reg_amps = off - reg_state_off;
        // register launches: pass p of every register-path circuit that has one
        std::vector<std::vector<int>> ta_of(b->count), op_of(b->count);
        for (int i : big_reg) {
            for (const qsv::TileProgram &pg : b->regplan[i].progs) {
                const size_t io = (imgs.size() + 255) & ~size_t(255);
                imgs.resize(io + pg.img.size());
                if (!pg.img.empty()) std::memcpy(imgs.data() + io, pg.img.data(), pg.img.size());
                img_max = std::max<uint32_t>(img_max, (uint32_t)((pg.img.size() + 15) & ~size_t(15)));
                ta_of[i].push_back((int)tas.size());
                op_of[i].push_back((int)rops.size());
                tas.push_back(reg_args(pg, b->nq[i], (int64_t)io));
                rops.insert(rops.end(), pg.rops.begin(), pg.rops.end());
            }
        }
        size_t p_reg = 0;
        for (int i : big_reg) p_reg = std::max(p_reg, b->regplan[i].progs.size());
        for (size_t p = 0; p < p_reg; ++p) {
            b->h_reg_seg_begin.push_back((int32_t)rsegs.size());
            uint64_t it = 0;
            int dg = 0;
            for (int i : big_reg) {
                if (b->regplan[i].progs.size() <= p) continue;
                qsv::dev::RegSeg sg{};
                sg.first = it;
                sg.state_off = state_off[i];
                sg.ta = ta_of[i][p];
                sg.op_begin = op_of[i][p];
                rsegs.push_back(sg);
                it += tas[sg.ta].n_tiles;
                if (!tas[sg.ta].no_diag) dg = 1;
            }
            b->h_reg_items.push_back(it);
            b->h_reg_dg.push_back(dg);
        }
        b->h_reg_seg_begin.push_back((int32_t)rsegs.size());
        for (int i : big_lds) n_pass_launches = std::max(n_pass_launches, circ[i].pass_count);
        for (int p = 0; p < n_pass_launches; ++p) {
            b->h_seg_begin.push_back((int32_t)segs.size());
            uint64_t it = 0;
            for (int i : big_lds) {
                if (circ[i].pass_count <= p) continue;
                qsv::dev::BatchSeg sg{};
                sg.first = it;
                sg.state_off = state_off[i];
                sg.pass = circ[i].pass_begin + p;
                sg.circuit = i;
                sg.init = p == 0 ? 1 : 0;
                segs.push_back(sg);
                it += 1ull << (b->nq[i] - passes[sg.pass].m);
            }
            b->h_items.push_back(it);
        }
        b->h_seg_begin.push_back((int32_t)segs.size());
        uint64_t it = 0;
        for (int i : big) {
            qsv::dev::BatchSeg sg{};
            sg.first = it;
            sg.state_off = state_off[i];
            sg.pass = -1;
            sg.circuit = i;
            segs.push_back(sg);
            const int cl = std::min(kChunkLog, b->nq[i]);
            it += 1ull << (b->nq[i] - cl);
        }
        b->h_items.push_back(it);
        b->h_seg_begin.push_back((int32_t)segs.size());
    }
    std::vector<int32_t> order;
    for (int i = 0; i < b->count; ++i)
        if (!pm || b->nq[i] <= mb) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    // matrices in the batch dtype
    std::vector<unsigned char> host;
    const size_t o_circ = put(host, circ);
    const size_t o_order = put(host, order);
    const size_t o_pass = put(host, passes);
    const size_t o_ops = put(host, tops);
    const size_t o_terms = put(host, terms);
    size_t o_pool;
    if (b->dtype == QSV_C128) {
        o_pool = put(host, mats);
    } else {
        std::vector<float> f(mats.begin(), mats.end());
        o_pool = put(host, f);
    }
    const size_t o_ctr = put(host, std::vector<uint32_t>(64, 0));
    const size_t o_out = put(host, std::vector<double>(b->count, 0.0));
    const size_t o_segs = put(host, segs);
    const size_t o_tas = put(host, tas);
    const size_t o_rops = put(host, rops);
    const size_t o_imgs = put(host, imgs);
    const size_t o_rsegs = put(host, rsegs);
    const size_t o_rstarts = put(host, reg_starts);
    const size_t o_part = put(host, std::vector<double>(pm ? b->h_items.back() : 1, 0.0));
    hipError_t e = hipMalloc(&b->d_buf, host.size());
    if (e != hipSuccess) return berr(QSV_ENOMEM, "hipMalloc of the batch plan failed");
    e = hipMemcpy(b->d_buf, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return berr(QSV_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    unsigned char *d = (unsigned char *)b->d_buf;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int occ = std::max(1, qsv::dev::batch_occupancy(b->dtype, mb, mfma_k));
    const unsigned grid = (unsigned)std::max(1, std::min(cus * occ, (int)order.size()));
    const uint64_t slot = max_big > 0 ? (1ull << max_big) : 1;
    if (pm && big_amps * elem > b->states_bytes) {
        if (b->d_states) (void)hipFree(b->d_states);
        b->d_states = nullptr;
        b->states_bytes = 0;
        e = hipMalloc(&b->d_states, big_amps * elem);
        if (e != hipSuccess) return berr(QSV_ENOMEM, "hipMalloc of the pass-major states failed");
        b->states_bytes = big_amps * elem;
    }
    const size_t need = (size_t)grid * slot * elem;
    if (need > b->scratch_bytes) {
        if (b->d_scratch) (void)hipFree(b->d_scratch);
        b->d_scratch = nullptr;
        b->scratch_bytes = 0;
        e = hipMalloc(&b->d_scratch, need);
        if (e != hipSuccess) return berr(QSV_ENOMEM, "hipMalloc of the batch scratch failed");
        b->scratch_bytes = need;
    }
    qsv::dev::BatchLaunch &L = b->L;
    L.circuits = (const qsv::dev::BatchCircuit *)(d + o_circ);
    L.order = (const int32_t *)(d + o_order);
    L.count = (int32_t)order.size();
    L.passes = (const qsv::dev::BatchPass *)(d + o_pass);
    L.ops = (const qsv::dev::TileOp *)(d + o_ops);
    L.pool = d + o_pool;
    L.terms = (const qsv::dev::BatchTerm *)(d + o_terms);
    L.scratch = b->d_scratch;
    L.slot_amps = slot;
    L.mb = mb;
    L.counter = (unsigned int *)(d + o_ctr);
    L.out = (double *)(d + o_out);
    L.grid = grid;
    L.mfma_k = mfma_k;
    L.pass_major = pm ? 1 : 0;
    L.n_pass_launches = pm ? n_pass_launches : 0;
    L.n_reg_launches = pm ? (int32_t)b->h_reg_items.size() : 0;
    L.reg_segs = (const qsv::dev::RegSeg *)(d + o_rsegs);
    L.reg_seg_begin = b->h_reg_seg_begin.data();
    L.reg_items = b->h_reg_items.data();
    L.reg_dg = b->h_reg_dg.data();
    L.tas = (const qsv::dev::TileArgs *)(d + o_tas);
    L.rops = (const qsv::dev::RegOp *)(d + o_rops);
    L.reg_pool = d + o_imgs;
    L.reg_img_max = img_max;
    L.reg_state_off = reg_state_off;
    L.reg_amps = reg_amps;
    L.reg_starts = (const uint64_t *)(d + o_rstarts);
    L.n_reg_states = (int32_t)reg_starts.size();
    L.segs = (const qsv::dev::BatchSeg *)(d + o_segs);
    L.seg_begin = b->h_seg_begin.data();
    L.items = b->h_items.data();
    L.states = b->d_states;
    L.partial = (double *)(d + o_part);
    L.chunk_log = kChunkLog;
    L.grid_big = (unsigned)(cus * std::max(1, qsv::dev::batch_pass_occupancy(b->dtype, mb, mfma_k)));
    b->mb = mb;
    b->kfuse = kf;
    if (b->use_graph) {
        e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = qsv::dev::batch_launch(b->dtype, L, b->stream);
            e = hipStreamEndCapture(b->stream, &b->graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return berr(QSV_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    return QSV_OK;
}

qsv_status launch(qsv_batch *b) {
    hipError_t e = hipEventRecord(b->e0, b->stream);
    if (e == hipSuccess)
        e = b->use_graph ? hipGraphLaunch(b->exec, b->stream)
                         : qsv::dev::batch_launch(b->dtype, b->L, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->e1, b->stream);
    if (e != hipSuccess) return berr(QSV_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
    return QSV_OK;
}

qsv_status timed_run(qsv_batch *b, double *ms) {
    qsv_status st = launch(b);
    if (st != QSV_OK) return st;
    hipError_t e = hipEventSynchronize(b->e1);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, b->e0, b->e1);
    if (e != hipSuccess) return berr(QSV_EDEVICE, std::string("batch run: ") + hipGetErrorString(e));
    *ms = f;
    return QSV_OK;
}

std::string cache_key(const qsv_batch *b) {
    int hist[31] = {};
    for (int n : b->nq) hist[n] += 1;
    std::ostringstream k;
    k << "gfx950/" << (b->dtype == QSV_C128 ? "c128" : "c64") << "/" << b->count << "/";
    for (int n = 1; n <= 30; ++n)
        if (hist[n]) k << n << ":" << hist[n] << ",";
    return k.str();
}

// tiny flat JSON object {"key": [mb, kf], ...}
std::map<std::string, std::pair<int, int>> read_cache(const char *path) {
    std::map<std::string, std::pair<int, int>> m;
    if (!path) return m;
    std::ifstream f(path);
    if (!f) return m;
    std::string s((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    size_t p = 0;
    while ((p = s.find('"', p)) != std::string::npos) {
        const size_t q = s.find('"', p + 1);
        if (q == std::string::npos) break;
        const std::string key = s.substr(p + 1, q - p - 1);
        int a = 0, c = 0;
        if (std::sscanf(s.c_str() + q + 1, " : [ %d , %d ]", &a, &c) == 2) m[key] = {a, c};
        p = q + 1;
    }
    return m;
}

void write_cache(const char *path, const std::map<std::string, std::pair<int, int>> &m) {
    if (!path) return;
    std::ofstream f(path);
    f << "{\n";
    size_t i = 0;
    for (const auto &kv : m)
        f << "  \"" << kv.first << "\": [" << kv.second.first << ", " << kv.second.second << "]"
          << (++i < m.size() ? ",\n" : "\n");
    f << "}\n";
}

}  // namespace

extern "C" {

qsv_status qsv_batch_create(int32_t count, const qsv_circuit *circuits, const qsv_pauli_sum *hams,
                            const qsv_batch_options *opt, qsv_batch **out) {
    if (!circuits || !hams || !opt || !out || count < 1) return berr(QSV_EINVAL, "bad argument");
    if (opt->dtype != QSV_C64 && opt->dtype != QSV_C128) return berr(QSV_EINVAL, "bad dtype");
    const int maxm = qsv::dev::tile_pass_max_bits(opt->dtype);
    if (opt->tile_bits < 0 || opt->tile_bits > maxm || (opt->tile_bits > 0 && opt->tile_bits < 8))
        return berr(QSV_EINVAL, "tile_bits must be 0 or 8.." + std::to_string(maxm));
    qsv_batch *b = new qsv_batch();
    b->count = count;
    b->dtype = opt->dtype;
    b->use_graph = opt->use_graph != 0;
    b->big_per_wg = opt->big_per_workgroup != 0;
    b->nq.resize(count);
    b->ops.resize(count);
    b->terms.resize(count);
    b->regplan.resize(count);
    for (int i = 0; i < count; ++i) {
        qsv_status st = parse(circuits[i], hams[i], i, b->ops[i], b->terms[i]);
        if (st != QSV_OK) {
            delete b;
            return st;
        }
        b->nq[i] = circuits[i].n_qubits;
    }
    hipError_t e = hipSuccess;
    if (opt->stream) {
        b->stream = (hipStream_t)opt->stream;
    } else {
        e = hipStreamCreate(&b->stream);   // graph capture needs a non-null stream
        b->own_stream = true;
    }
    if (e == hipSuccess) e = hipEventCreate(&b->e0);
    if (e == hipSuccess) e = hipEventCreate(&b->e1);
    if (e != hipSuccess) {
        qsv_batch_destroy(b);
        return berr(QSV_EDEVICE, std::string("stream/event: ") + hipGetErrorString(e));
    }
    int mb = opt->tile_bits > 0 ? opt->tile_bits : (opt->dtype == QSV_C128 ? 11 : 12);
    int kf = 2;
    if (opt->autotune && opt->tile_bits == 0) {
        auto cache = read_cache(opt->tune_cache);
        const std::string key = cache_key(b);
        auto it = cache.find(key);
        if (it != cache.end()) {
            mb = it->second.first;
            kf = it->second.second;
        } else {
            double best = 1e300;
            const int mbs_c64[] = {11, 12, 13};
            const int mbs_c128[] = {10, 11, 12};
            const int *mbs = opt->dtype == QSV_C128 ? mbs_c128 : mbs_c64;
            for (int a = 0; a < 3; ++a)
                for (int kk = 1; kk <= 3; ++kk) {
                    qsv_status st = build_plan(b, mbs[a], kk);
                    double ms = 0, ms2 = 0;
                    if (st == QSV_OK) st = timed_run(b, &ms);
                    if (st == QSV_OK) st = timed_run(b, &ms2);
                    if (st != QSV_OK) {
                        qsv_batch_destroy(b);
                        return st;
                    }
                    if (ms2 < best) {
                        best = ms2;
                        mb = mbs[a];
                        kf = kk;
                    }
                }
            cache[key] = {mb, kf};
            write_cache(opt->tune_cache, cache);
        }
    }
    qsv_status st = build_plan(b, mb, kf);
    if (st != QSV_OK) {
        qsv_batch_destroy(b);
        return st;
    }
    *out = b;
    return QSV_OK;
}

qsv_status qsv_batch_run(qsv_batch *b, double *out_host) {
    if (!b || !out_host) return berr(QSV_EINVAL, "bad argument");
    qsv_status st = launch(b);
    if (st != QSV_OK) return st;
    hipError_t e = hipMemcpyAsync(out_host, b->L.out, sizeof(double) * b->count,
                                  hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, b->e0, b->e1);
    if (e != hipSuccess) return berr(QSV_EDEVICE, std::string("batch run: ") + hipGetErrorString(e));
    b->last_ms = f;
    return QSV_OK;
}

qsv_status qsv_batch_info(const qsv_batch *b, int32_t *tile_bits, int32_t *k_fuse,
                          double *last_ms) {
    if (!b) return berr(QSV_EINVAL, "NULL batch");
    if (tile_bits) *tile_bits = b->mb;
    if (k_fuse) *k_fuse = b->kfuse;
    if (last_ms) *last_ms = b->last_ms;
    return QSV_OK;
}

qsv_status qsv_batch_destroy(qsv_batch *b) {
    if (!b) return QSV_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    free_plan(b);
    if (b->d_scratch) (void)hipFree(b->d_scratch);
    if (b->d_states) (void)hipFree(b->d_states);
    if (b->e0) (void)hipEventDestroy(b->e0);
    if (b->e1) (void)hipEventDestroy(b->e1);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return QSV_OK;
}

}  // extern "C"
