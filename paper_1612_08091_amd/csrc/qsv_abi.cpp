// C-ABI entry points of libqsv and the runtime behind them: handle, qubit-id
// map, lazy gate queue, flush dispatch (per gate / fused / LDS-tile passes),
// reductions, measurement, (de)allocation.
//
// Device memory for the state is materialised lazily: until a call needs the
// amplitudes on the device, a handle only records that its state is |0...0>.
// So creating handles, allocating qubits, queueing gates and planning work
// without a GPU, which keeps argument validation testable on a CPU host.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/qsv.h"
#include "adjoint_tile.hpp"
#include "device.hpp"
#include "dm.hpp"
#include "math_gate.hpp"
#include "qsv_internal.hpp"
#include "tileprog.hpp"

using qsv::cd;
using qsv::Gate;
using qsv::Op;
using qsv::Pass;
using qsv::popc;

struct qsv_sim {
    qsv_options opt{};
    int n = 0;
    std::vector<int> id_at;            // bit position -> qubit id
    int pos_of[64];                    // qubit id -> bit position, -1 if free
    std::vector<Gate> queue;
    bool materialized = false;         // device buffer holds the state
    bool invalid = false;              // a flush failed after enqueueing kernels
    int64_t inject_fail_at = -1;       // tests of error handling: launch number that fails
    int64_t launches_seen = 0;
    void *d_state = nullptr;
    bool owns_state = false;
    uint64_t cap_amps = 0;             // amplitudes the device buffer holds
    hipStream_t stream = nullptr;
    std::string err;
    qsv_stats stats{};
    uint64_t stats_remaps = 0;
    // workspace for reductions
    void *d_ws = nullptr;
    size_t ws_bytes = 0;
    double *d_small = nullptr;         // 16 doubles
    // op pool for tile passes: pinned host staging + device copy, two slots
    struct Slot {
        void *h = nullptr;
        void *d = nullptr;
        size_t bytes = 0;
        hipEvent_t done = nullptr;
        bool pending = false;
    } slot[2];
    int cur_slot = 0;
    // kernel timing (opt.timing): events bracketing launches
    struct EvRec {
        hipEvent_t a, b;
        int cls;
        double bytes;
    };
    std::vector<EvRec> ev_pending;
    std::vector<hipEvent_t> ev_pool;
    double k_ms[QSV_K_COUNT] = {0, 0, 0, 0};
    uint64_t k_launch[QSV_K_COUNT] = {0, 0, 0, 0};
    double k_bytes[QSV_K_COUNT] = {0, 0, 0, 0};
    // second state buffer of the math gates (same capacity as the state)
    void *d_alt = nullptr;
    uint64_t alt_amps = 0;
    // adjoint / scratch vectors
    void *d_vec[3] = {nullptr, nullptr, nullptr};
    uint64_t vec_amps = 0;
    int vec_dtype = -1;

    int elem() const { return opt.dtype == QSV_C128 ? 16 : 8; }
    uint64_t dim() const { return 1ull << n; }
};

namespace {

std::mutex g_mu;
std::unordered_set<const qsv_sim *> g_live;
thread_local std::string g_err;

bool live(const qsv_sim *s) {
    std::lock_guard<std::mutex> lk(g_mu);
    return s && g_live.count(s);
}

qsv_status fail(qsv_sim *s, qsv_status st, const std::string &msg) {
    if (s) s->err = msg;
    else g_err = msg;
    return st;
}

qsv_status hip_fail(qsv_sim *s, hipError_t e, const char *where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(s, QSV_EDEVICE, m);
}

#define QSV_HIP(s, call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail((s), e_, #call); \
    } while (0)

#define QSV_TRY(expr)                      \
    do {                                   \
        qsv_status st_ = (expr);           \
        if (st_ != QSV_OK) return st_;     \
    } while (0)

#define QSV_CHECK(s)                                                              \
    do {                                                                          \
        if (!live(s)) return fail(nullptr, QSV_ESTATE, "invalid or destroyed handle"); \
        (s)->err.clear();                                                         \
    } while (0)

// 4096-amplitude tiles (256 threads x 16 amplitudes) for both dtypes: 32 KiB
// (complex128) or 16 KiB (complex64) of LDS for the two-phase remaps.
int default_tile_bits(int) { return 12; }

// QSV_LOG environment variable: 0 silent (default), 1 flush summaries,
// 2 one line per planned pass, on stderr.
int log_level() {
    static int lvl = -1;
    if (lvl < 0) {
        const char *e = std::getenv("QSV_LOG");
        lvl = e ? std::atoi(e) : 0;
    }
    return lvl;
}

// ------------------------------------------------------------- device memory
qsv_status ensure_capacity(qsv_sim *s, int nq) {
    const uint64_t need = 1ull << nq;
    if (need <= s->cap_amps) return QSV_OK;
    if (!s->owns_state && s->d_state)
        return fail(s, QSV_ENOMEM, "borrowed state buffer too small");
    uint64_t amps = std::max<uint64_t>(need, 1024);
    const uint64_t bytes = amps * s->elem();
    // decided before allocating: against the handle's limit when it has one
    // (no device call), else against the device's free memory
    if (s->opt.mem_limit != 0) {
        if (bytes > s->opt.mem_limit)
            return fail(s, QSV_ENOMEM, "the state needs " + std::to_string(bytes) +
                                           " bytes, over the handle's mem_limit of " +
                                           std::to_string(s->opt.mem_limit));
    } else {
        size_t free_b = 0, total_b = 0;
        QSV_HIP(s, hipMemGetInfo(&free_b, &total_b));
        if (bytes > free_b)
            return fail(s, QSV_ENOMEM, "the state needs " + std::to_string(bytes) +
                                           " bytes, the device has " + std::to_string(free_b) +
                                           " free of " + std::to_string(total_b));
    }
    void *nb = nullptr;
    hipError_t e = hipMalloc(&nb, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            return fail(s, QSV_ENOMEM, "hipMalloc of the state failed (out of device memory)");
        return hip_fail(s, e, "hipMalloc of the state");
    }
    if (s->d_state && s->materialized)
        QSV_HIP(s, hipMemcpyAsync(nb, s->d_state, s->dim() * s->elem(), hipMemcpyDeviceToDevice,
                                  s->stream));
    if (s->d_state) {
        QSV_HIP(s, hipStreamSynchronize(s->stream));
        QSV_HIP(s, hipFree(s->d_state));
    }
    s->d_state = nb;
    s->cap_amps = amps;
    s->owns_state = true;
    return QSV_OK;
}

qsv_status invalid_state(qsv_sim *s) {
    return fail(s, QSV_EDEVICE,
                "the state is invalid after a flush that failed part way; call qsv_reset or "
                "qsv_set_state");
}

qsv_status materialize(qsv_sim *s) {
    if (s->invalid) return invalid_state(s);
    if (s->materialized) return QSV_OK;
    QSV_TRY(ensure_capacity(s, s->n));
    QSV_HIP(s, qsv::dev::fill_basis0(s->opt.dtype, s->d_state, s->dim(), s->stream));
    if (!s->d_small) QSV_HIP(s, hipMalloc((void **)&s->d_small, 64 * sizeof(double)));
    s->materialized = true;
    return QSV_OK;
}

qsv_status ensure_ws(qsv_sim *s, size_t bytes) {
    if (bytes <= s->ws_bytes) return QSV_OK;
    if (s->d_ws) {
        QSV_HIP(s, hipStreamSynchronize(s->stream));
        QSV_HIP(s, hipFree(s->d_ws));
        s->d_ws = nullptr;
        s->ws_bytes = 0;
    }
    size_t b = std::max<size_t>(bytes, 1 << 20);
    QSV_HIP(s, hipMalloc(&s->d_ws, b));
    s->ws_bytes = b;
    return QSV_OK;
}

// Stage `bytes` of host data into the current pool slot; returns the device
// pointer.  The slot's previous upload must have completed before its host
// buffer is overwritten.
qsv_status stage(qsv_sim *s, const void *data, size_t bytes, void **dptr) {
    qsv_sim::Slot &sl = s->slot[s->cur_slot];
    s->cur_slot ^= 1;
    if (sl.pending) {
        QSV_HIP(s, hipEventSynchronize(sl.done));
        sl.pending = false;
    }
    if (bytes > sl.bytes) {
        QSV_HIP(s, hipStreamSynchronize(s->stream));
        if (sl.h) QSV_HIP(s, hipHostFree(sl.h));
        if (sl.d) QSV_HIP(s, hipFree(sl.d));
        sl.h = sl.d = nullptr;
        size_t b = std::max<size_t>(bytes, 1 << 20);
        QSV_HIP(s, hipHostMalloc(&sl.h, b, hipHostMallocDefault));
        QSV_HIP(s, hipMalloc(&sl.d, b));
        sl.bytes = b;
        if (!sl.done) QSV_HIP(s, hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    }
    std::memcpy(sl.h, data, bytes);
    QSV_HIP(s, hipMemcpyAsync(sl.d, sl.h, bytes, hipMemcpyHostToDevice, s->stream));
    QSV_HIP(s, hipEventRecord(sl.done, s->stream));
    sl.pending = true;
    *dptr = sl.d;
    return QSV_OK;
}

// ------------------------------------------------------------------ timing
hipEvent_t pool_event(qsv_sim *s) {
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Record the start of a launch; returns an opaque token (or -1).
int tbegin(qsv_sim *s) {
    if (!s->opt.timing) return -1;
    hipEvent_t a = pool_event(s), b = pool_event(s);
    if (!a || !b) return -1;
    if (hipEventRecord(a, s->stream) != hipSuccess) return -1;
    s->ev_pending.push_back({a, b, 0, 0.0});
    return (int)s->ev_pending.size() - 1;
}

void tend(qsv_sim *s, int tok, int cls, double bytes) {
    if (tok < 0) return;
    auto &r = s->ev_pending[tok];
    r.cls = cls;
    r.bytes = bytes;
    (void)hipEventRecord(r.b, s->stream);
}

qsv_status collect_times(qsv_sim *s) {
    for (auto &r : s->ev_pending) {
        QSV_HIP(s, hipEventSynchronize(r.b));
        float ms = 0.f;
        QSV_HIP(s, hipEventElapsedTime(&ms, r.a, r.b));
        s->k_ms[r.cls] += ms;
        s->k_launch[r.cls] += 1;
        s->k_bytes[r.cls] += r.bytes;
        s->ev_pool.push_back(r.a);
        s->ev_pool.push_back(r.b);
    }
    s->ev_pending.clear();
    return QSV_OK;
}

// --------------------------------------------------------------- launching
void index_args(uint64_t insert_mask, uint64_t ones, qsv::dev::IndexArgs &ia) {
    ia.npos = 0;
    for (int p = 0; p < 64; ++p)
        if ((insert_mask >> p) & 1) ia.pos[ia.npos++] = (uint8_t)p;
    ia.ones = ones;
}

uint64_t offset_of(int r, const int *t, int k) {
    uint64_t o = 0;
    for (int j = 0; j < k; ++j)
        if ((r >> j) & 1) o |= 1ull << t[j];
    return o;
}

void account(qsv_sim *s, double touched_amps, double flops_per_amp) {
    s->stats.kernels += 1;
    s->stats.passes += 1;
    s->stats.alg_bytes += 2.0 * touched_amps * s->elem();
    s->stats.alg_flops += touched_amps * flops_per_amp;
}

qsv_status run_tile_passes(qsv_sim *s, const std::vector<Pass> &passes);
std::vector<Pass> plan_flush(const qsv_sim *s, const std::vector<Op> &ops, int m);

// Register bits per thread of the register-resident tile kernel.
int reg_bits_for(const qsv_sim *s) {
    if (s->opt.reg_bits > 0) return s->opt.reg_bits;
    if (s->opt.tile_bits >= 11 && s->opt.tile_bits <= 13) return s->opt.tile_bits - 8;
    return qsv::dev::tile_reg_bits(s->opt.dtype);
}

// Every kernel launch of a flush passes here first.  QSV_INJECT_LAUNCH_FAILURE=k
// (read at qsv_create; for tests of error handling) makes launch number k of
// the handle fail as a device error would, without launching it.
qsv_status launch_gate(qsv_sim *s) {
    if (s->inject_fail_at >= 0 && s->launches_seen++ == s->inject_fail_at)
        return fail(s, QSV_EDEVICE, "injected launch failure");
    return QSV_OK;
}

qsv_status launch_op(qsv_sim *s, const Op &op) {
    QSV_TRY(launch_gate(s));
    const int nq = s->n;
    const int k = op.k;
    const int c = popc(op.ctrl);
    const uint64_t ngroups = 1ull << (nq - k - c);
    qsv::dev::IndexArgs ia;
    index_args(op.targets() | op.ctrl, op.ctrl, ia);
    if (op.kind == Op::MONO) {
        if (op.touch == 0) return QSV_OK;
        qsv::dev::MonoArgs a{};
        for (int r = 0; r < (1 << k); ++r) {
            a.vr[r] = op.U[r].real();
            a.vi[r] = op.U[r].imag();
            a.off[r] = offset_of(r, op.t, k);
            a.srcoff[r] = offset_of(op.perm[r], op.t, k);
        }
        a.touch = op.touch;
        const double touched = (double)popc(op.touch) * (double)ngroups;
        const int tok = tbegin(s);
        QSV_HIP(s, qsv::dev::launch_mono(s->opt.dtype, s->d_state, k, ngroups, ia, a, s->stream));
        tend(s, tok, QSV_K_MONO, 2.0 * touched * s->elem());
        bool pure_perm = true;
        for (int r = 0; r < (1 << k); ++r)
            if (op.U[r] != cd(1, 0)) pure_perm = false;
        account(s, touched, pure_perm ? 0.0 : 6.0);
        return QSV_OK;
    }
    if (k <= 3) {
        qsv::dev::DenseArgs a{};
        const int D = 1 << k;
        for (int i = 0; i < D * D; ++i) {
            a.mr[i] = op.U[i].real();
            a.mi[i] = op.U[i].imag();
        }
        for (int r = 0; r < D; ++r) a.off[r] = offset_of(r, op.t, k);
        const int tok = tbegin(s);
        QSV_HIP(s, qsv::dev::launch_dense(s->opt.dtype, s->d_state, k, ngroups, ia, a, s->stream));
        tend(s, tok, QSV_K_DENSE, 2.0 * (double)(ngroups << k) * s->elem());
        account(s, (double)(ngroups << k), 8.0 * D - 2.0);
        return QSV_OK;
    }
    // k = 4, 5: one LDS-tile pass holding this op only
    std::vector<Pass> one(1);
    int m = s->opt.tile_bits > 0 ? s->opt.tile_bits : default_tile_bits(s->opt.dtype);
    m = std::min(m, nq);
    uint64_t tile = op.targets();
    for (int p = 0; p < nq && popc(tile) < m; ++p) tile |= 1ull << p;
    one[0].tile = tile;
    one[0].ops.push_back(op);
    return run_tile_passes(s, one);
}

// Lower every pass (register-resident kernel when the tile has RB + 8 bits,
// LDS kernel otherwise), upload all descriptors and matrices in one copy,
// then launch one tile kernel per pass.
qsv_status run_tile_passes(qsv_sim *s, const std::vector<Pass> &passes) {
    using qsv::dev::RegOp;
    using qsv::dev::TileOp;
    const int nq = s->n;
    const int rb = reg_bits_for(s);
    std::vector<double> mats;
    std::vector<qsv::TileProgram> progs(passes.size());
    size_t n_rops = 0, n_lops = 0;
    {
        // Passes lower independently, on several host threads when there
        // are many (the GPU waits for the programs): each into its own
        // matrix list, then the lists are joined and the LDS ops' matrix
        // offsets moved by their pass's start.
        std::vector<std::vector<double>> pm(passes.size());
        auto work = [&](size_t pi) {
            qsv::compile_pass(passes[pi], rb, pm[pi], progs[pi], (int)s->elem());
        };
        const unsigned hw = std::thread::hardware_concurrency();
        const size_t nth = passes.size() < 4 ? 1 : std::min<size_t>(passes.size(), std::min(8u, std::max(1u, hw)));
        if (nth <= 1) {
            for (size_t pi = 0; pi < passes.size(); ++pi) work(pi);
        } else {
            std::atomic<size_t> next{0};
            std::vector<std::thread> th;
            th.reserve(nth);
            for (size_t t = 0; t < nth; ++t)
                th.emplace_back([&]() {
                    for (size_t i; (i = next.fetch_add(1)) < passes.size();) work(i);
                });
            for (std::thread &x : th) x.join();
        }
        for (size_t pi = 0; pi < passes.size(); ++pi) {
            const int64_t base = (int64_t)(mats.size() / 2);
            for (qsv::dev::TileOp &t : progs[pi].lops) t.mat += base;
            mats.insert(mats.end(), pm[pi].begin(), pm[pi].end());
            n_rops += progs[pi].rops.size();
            n_lops += progs[pi].lops.size();
        }
    }
    // pool: [RegOp array][TileOp array][one zeroed tile counter per pass]
    //       [matrices in the state dtype][LDS images of the register passes]
    const size_t r_bytes = (n_rops * sizeof(RegOp) + 255) & ~size_t(255);
    const size_t l_bytes = (n_lops * sizeof(TileOp) + 255) & ~size_t(255);
    const size_t c_bytes = (passes.size() * sizeof(unsigned int) + 255) & ~size_t(255);
    const size_t nmat = mats.size();
    const size_t mat_bytes =
        ((s->opt.dtype == QSV_C128 ? nmat * sizeof(double) : nmat * sizeof(float)) + 255) &
        ~size_t(255);
    std::vector<size_t> img_at(passes.size(), 0);
    size_t img_bytes = 0;
    for (size_t pi = 0; pi < passes.size(); ++pi) {
        img_at[pi] = mat_bytes + img_bytes;   // relative to the matrices
        img_bytes += (progs[pi].img.size() + 255) & ~size_t(255);
    }
    std::vector<unsigned char> host(r_bytes + l_bytes + c_bytes + mat_bytes + img_bytes + 16, 0);
    {
        size_t ro = 0, lo = 0;
        for (const auto &pg : progs) {
            if (!pg.rops.empty())
                std::memcpy(host.data() + ro * sizeof(RegOp), pg.rops.data(), pg.rops.size() * sizeof(RegOp));
            if (!pg.lops.empty())
                std::memcpy(host.data() + r_bytes + lo * sizeof(TileOp), pg.lops.data(),
                            pg.lops.size() * sizeof(TileOp));
            ro += pg.rops.size();
            lo += pg.lops.size();
        }
    }
    for (size_t pi = 0; pi < passes.size(); ++pi)
        if (!progs[pi].img.empty())
            std::memcpy(host.data() + r_bytes + l_bytes + c_bytes + img_at[pi], progs[pi].img.data(),
                        progs[pi].img.size());
    if (s->opt.dtype == QSV_C128) {
        if (nmat) std::memcpy(host.data() + r_bytes + l_bytes + c_bytes, mats.data(), nmat * sizeof(double));
    } else {
        float *f = reinterpret_cast<float *>(host.data() + r_bytes + l_bytes + c_bytes);
        for (size_t i = 0; i < nmat; ++i) f[i] = (float)mats[i];
    }
    void *dpool = nullptr;
    QSV_TRY(stage(s, host.data(), host.size(), &dpool));
    const RegOp *drops = reinterpret_cast<const RegOp *>(dpool);
    const TileOp *dlops = reinterpret_cast<const TileOp *>((const unsigned char *)dpool + r_bytes);
    unsigned int *dcount = reinterpret_cast<unsigned int *>((unsigned char *)dpool + r_bytes + l_bytes);
    const void *dmat = (const unsigned char *)dpool + r_bytes + l_bytes + c_bytes;
    size_t ro = 0, lo = 0;
    for (size_t pi = 0; pi < passes.size(); ++pi) {
        const qsv::TileProgram &pg = progs[pi];
        const size_t nr = pg.rops.size(), nl = pg.lops.size();
        if (((pg.reg && nr == 0) || (!pg.reg && nl == 0)) && !pg.permutes) {
            ro += nr;
            lo += nl;
            continue;
        }
        QSV_TRY(launch_gate(s));
        qsv::dev::TileArgs ta{};
        ta.m = pg.m;
        ta.nq = nq;
        ta.tile_pos_n = pg.m;
        int c = 0;
        for (int p = 0; p < 64; ++p)
            if ((pg.tile >> p) & 1) ta.tpos[c++] = (uint32_t)p;
        ta.n_tiles = 1ull << (nq - pg.m);
        std::memcpy(ta.g_reg, pg.g_reg, sizeof(ta.g_reg));
        std::memcpy(ta.g_thr, pg.g_thr, sizeof(ta.g_thr));
        std::memcpy(ta.g_reg_f, pg.g_reg_f, sizeof(ta.g_reg_f));
        std::memcpy(ta.g_thr_f, pg.g_thr_f, sizeof(ta.g_thr_f));
        ta.img_bytes = (uint32_t)pg.img.size();
        ta.store_sync = pg.store_sync ? 1 : 0;
        ta.img_off = (int64_t)img_at[pi];
        ta.rb = rb;
        ta.mfma_k = pg.mfma_k;
        for (int b = 0; b < pg.m; ++b) ta.spos[b] = pg.spos[b];
        for (int i = 0; i < 64 && (i << 8) < (1 << pg.m); ++i) {
            uint64_t d = 0, f = 0;
            for (int b = 8; b < pg.m; ++b)
                if (((i << 8) >> b) & 1) {
                    d |= 1ull << ta.tpos[b];
                    f |= 1ull << ta.spos[b];
                }
            ta.dep_hi[i] = d;
            ta.dep_hi_f[i] = f;
        }
        const int tok = tbegin(s);
        if (pg.reg) {
            ta.n_ops = (int)nr;
            ta.no_diag = 1;
            for (const qsv::dev::RegOp &r : pg.rops)
                if (r.kind == qsv::dev::ROP_DIAG) ta.no_diag = 0;
            QSV_HIP(s, qsv::dev::launch_tile_reg(s->opt.dtype, s->d_state, ta, drops + ro, dmat,
                                                 dcount + pi, s->stream));
        } else {
            ta.n_ops = (int)nl;
            QSV_HIP(s, qsv::dev::launch_tile_pass(s->opt.dtype, s->d_state, ta, dlops + lo, dmat,
                                                  dcount + pi, s->stream));
        }
        tend(s, tok, QSV_K_TILE, 2.0 * (double)s->dim() * s->elem());
        account(s, (double)s->dim(), pg.flops_per_amp);
        if (log_level() >= 2)
            std::fprintf(stderr,
                         "qsv: pass %zu tile=%#llx m=%d %s ops=%zu remaps=%d real=%d diag=%d "
                         "image=%zuB flop/amp=%.0f\n",
                         pi, (unsigned long long)pg.tile, pg.m, pg.reg ? "reg" : "lds",
                         pg.reg ? nr - pg.remaps : nl, pg.remaps, pg.real_ops, pg.diag_ops,
                         pg.img.size(), pg.flops_per_amp);
        s->stats_remaps += pg.remaps;
        ro += nr;
        lo += nl;
    }
    return QSV_OK;
}

int tile_bits_for(const qsv_sim *s) {
    int m = s->opt.tile_bits > 0 ? s->opt.tile_bits : default_tile_bits(s->opt.dtype);
    return std::min(m, qsv::dev::tile_pass_max_bits(s->opt.dtype));
}

// Tiled plan of a flush.  The page bit is the amplitude index bit of a 2 MiB
// page: 17 for 16-byte amplitudes, 18 for 8-byte ones.
std::vector<Pass> plan_flush(const qsv_sim *s, const std::vector<Op> &ops, int m) {
    const int page_bit = s->elem() == 16 ? 17 : 18;
    return qsv::plan_tiled(ops, s->n, m, s->opt.k_max, page_bit, s->opt.relabel != 0);
}

std::vector<Op> canonical_queue(const qsv_sim *s, uint64_t *dropped) {
    std::vector<Op> ops;
    ops.reserve(s->queue.size());
    uint64_t drop = 0;
    for (const Gate &g : s->queue) {
        Op op;
        if (qsv::canonicalize(g, op)) ops.push_back(std::move(op));
        else ++drop;
    }
    if (dropped) *dropped = drop;
    return ops;
}

qsv_status do_flush(qsv_sim *s) {
    if (s->invalid) return invalid_state(s);
    if (s->queue.empty()) return QSV_OK;
    QSV_TRY(materialize(s));
    std::vector<Op> ops = canonical_queue(s, nullptr);
    const uint64_t kernels0 = s->stats.kernels;
    auto run = [&]() -> qsv_status {
        const int mode = s->opt.mode;
        if (mode == QSV_MODE_PERGATE) {
            s->stats.fused_ops += ops.size();
            for (const Op &op : ops) QSV_TRY(launch_op(s, op));
        } else if (mode == QSV_MODE_FUSED) {
            std::vector<Op> f = qsv::fuse(ops, s->opt.k_max);
            s->stats.fused_ops += f.size();
            for (const Op &op : f) QSV_TRY(launch_op(s, op));
        } else {
            const int m = std::min(tile_bits_for(s), s->n);
            std::vector<Pass> passes = plan_flush(s, ops, m);
            for (const Pass &p : passes) s->stats.fused_ops += p.ops.size();
            QSV_TRY(run_tile_passes(s, passes));
        }
        return QSV_OK;
    };
    const qsv_status st = run();
    if (st != QSV_OK) {
        // Kernels already enqueued have changed the state: applying the queue
        // again would apply those gates twice.  Drop it and refuse the state
        // until it is reset or set.  With nothing enqueued the queue stays.
        if (s->stats.kernels != kernels0) {
            s->queue.clear();
            s->invalid = true;
            s->err += " (after " + std::to_string(s->stats.kernels - kernels0) +
                      " kernels of the flush ran: the queue is dropped and the state is invalid "
                      "until qsv_reset or qsv_set_state)";
        }
        return st;
    }
    s->stats.gates += s->queue.size();
    s->stats.amp_gate_updates += (double)s->queue.size() * (double)s->dim();
    s->queue.clear();
    return QSV_OK;
}

qsv_status sync(qsv_sim *s) {
    QSV_HIP(s, hipStreamSynchronize(s->stream));
    return QSV_OK;
}

qsv_status check_ids(qsv_sim *s, int32_t m, const int32_t *ids, uint64_t *mask_out) {
    uint64_t mask = 0;
    for (int j = 0; j < m; ++j) {
        const int id = ids[j];
        if (id < 0 || id >= 64 || s->pos_of[id] < 0)
            return fail(s, QSV_EINVAL, "unknown qubit id " + std::to_string(id));
        const uint64_t b = 1ull << s->pos_of[id];
        if (mask & b) return fail(s, QSV_EINVAL, "qubit id repeated: " + std::to_string(id));
        mask |= b;
    }
    if (mask_out) *mask_out = mask;
    return QSV_OK;
}

qsv_status prob_split_host(qsv_sim *s, int pos, double *p0, double *p1) {
    QSV_TRY(ensure_ws(s, qsv::dev::reduce_workspace_bytes(s->n)));
    const int tok = tbegin(s);
    QSV_HIP(s, qsv::dev::prob_split(s->opt.dtype, s->d_state, s->n, pos, (double *)s->d_ws,
                                    s->d_small, s->stream));
    tend(s, tok, QSV_K_REDUCE, (double)s->dim() * s->elem());
    double h[2];
    QSV_HIP(s, hipMemcpyAsync(h, s->d_small, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    QSV_TRY(sync(s));
    *p0 = h[0];
    *p1 = h[1];
    s->stats.kernels += 2;
    s->stats.alg_bytes += (double)s->dim() * s->elem();
    return QSV_OK;
}

}  // namespace

void qsv::set_last_error(const std::string &msg) { g_err = msg; }

// =================================================================== ABI
// ----------------------------------------------------------- density matrices
namespace {

// Validate system qubit indices of a density-matrix call; n = live / 2.
qsv_status dm_check(qsv_sim *s, int k, const int32_t *targets, int c, const int32_t *controls,
                    int kmax, uint64_t *tmask, uint64_t *cmask) {
    if ((s->n & 1) || s->n == 0)
        return fail(s, QSV_EINVAL, "a density matrix needs an even, nonzero number of qubits");
    const int n = s->n / 2;
    if (!targets || (c > 0 && !controls)) return fail(s, QSV_EINVAL, "NULL argument");
    if (k < 1 || k > kmax) return fail(s, QSV_EINVAL, "unsupported number of targets");
    if (c < 0 || k + c > n) return fail(s, QSV_EINVAL, "too many qubits");
    uint64_t seen = 0;
    *tmask = *cmask = 0;
    for (int j = 0; j < k + c; ++j) {
        const int q = j < k ? targets[j] : controls[j - k];
        if (q < 0 || q >= n || ((seen >> q) & 1))
            return fail(s, QSV_EINVAL, "system qubit index out of range or repeated");
        seen |= 1ull << q;
        (j < k ? *tmask : *cmask) |= 1ull << q;
    }
    return QSV_OK;
}

void dm_queue(qsv_sim *s, Gate &&g) {
    s->queue.push_back(std::move(g));
}

}  // namespace

extern "C" {

const char *qsv_version(void) { return "qsv 0.1 (gfx950)"; }

qsv_status qsv_copy_probe(const void *src, void *dst, uint64_t bytes, void *stream) {
    if (!src || !dst || bytes % 16) return fail(nullptr, QSV_EINVAL, "copy probe: NULL buffer or size not a multiple of 16");
    const hipError_t e = qsv::dev::copy_probe(src, dst, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, QSV_EDEVICE, std::string("copy probe: ") + hipGetErrorString(e));
    return QSV_OK;
}

const char *qsv_last_error(const qsv_sim *sim) {
    if (sim && live(sim)) return sim->err.c_str();
    return g_err.c_str();
}

qsv_status qsv_options_default(qsv_options *opt) {
    if (!opt) return fail(nullptr, QSV_EINVAL, "NULL options");
    std::memset(opt, 0, sizeof(*opt));
    opt->n_max = 30;
    opt->dtype = QSV_C128;
    opt->mode = QSV_MODE_TILED;
    opt->k_max = 2;
    opt->tile_bits = 0;
    opt->queue_limit = 0;
    opt->relabel = 1;
    return QSV_OK;
}

qsv_status qsv_create(const qsv_options *opt, qsv_sim **out) {
    if (!opt || !out) return fail(nullptr, QSV_EINVAL, "NULL argument");
    if (opt->n_max < 1 || opt->n_max > qsv::kMaxQubits)
        return fail(nullptr, QSV_EINVAL, "n_max must be in 1..36");
    if (opt->dtype != QSV_C128 && opt->dtype != QSV_C64)
        return fail(nullptr, QSV_EINVAL, "dtype must be QSV_C128 or QSV_C64");
    if (opt->mode < QSV_MODE_PERGATE || opt->mode > QSV_MODE_TILED)
        return fail(nullptr, QSV_EINVAL, "unknown mode");
    if (opt->mode != QSV_MODE_PERGATE && (opt->k_max < 1 || opt->k_max > qsv::kMaxK))
        return fail(nullptr, QSV_EINVAL, "k_max must be in 1..5");
    const int maxm = qsv::dev::tile_pass_max_bits(opt->dtype);
    if (opt->tile_bits < 0 || opt->tile_bits > maxm ||
        (opt->tile_bits > 0 && opt->tile_bits < qsv::kMaxK + 1))
        return fail(nullptr, QSV_EINVAL, "tile_bits must be 0 or in 6.." + std::to_string(maxm));
    if (opt->queue_limit < 0) return fail(nullptr, QSV_EINVAL, "queue_limit must be >= 0");
    if (opt->timing != 0 && opt->timing != 1) return fail(nullptr, QSV_EINVAL, "timing must be 0 or 1");
    if (opt->reg_bits != 0 && (opt->reg_bits < 3 || opt->reg_bits > 5))
        return fail(nullptr, QSV_EINVAL, "reg_bits must be 0 or 3..5");
    if (opt->relabel != 0 && opt->relabel != 1)
        return fail(nullptr, QSV_EINVAL, "relabel must be 0 or 1");
    const int elem = opt->dtype == QSV_C128 ? 16 : 8;
    if (opt->state) {
        if (opt->state_bytes < (uint64_t)elem << opt->n_max)
            return fail(nullptr, QSV_ENOMEM, "borrowed state buffer smaller than 2^n_max amplitudes");
    }
    qsv_sim *s = new qsv_sim();
    s->opt = *opt;
    s->stream = (hipStream_t)opt->stream;
    if (const char *e = std::getenv("QSV_INJECT_LAUNCH_FAILURE")) s->inject_fail_at = std::atoll(e);
    for (int i = 0; i < 64; ++i) s->pos_of[i] = -1;
    if (opt->state) {
        s->d_state = opt->state;
        s->owns_state = false;
        s->cap_amps = opt->state_bytes / elem;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(s);
    }
    *out = s;
    return QSV_OK;
}

qsv_status qsv_destroy(qsv_sim *s) {
    if (!s) return QSV_OK;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_live.count(s)) return fail(nullptr, QSV_ESTATE, "invalid or destroyed handle");
        g_live.erase(s);
    }
    if (s->materialized || s->d_ws || s->slot[0].h || s->slot[1].h) (void)hipStreamSynchronize(s->stream);
    if (s->owns_state && s->d_state) (void)hipFree(s->d_state);
    if (s->d_ws) (void)hipFree(s->d_ws);
    if (s->d_alt) (void)hipFree(s->d_alt);
    if (s->d_small) (void)hipFree(s->d_small);
    for (auto &sl : s->slot) {
        if (sl.h) (void)hipHostFree(sl.h);
        if (sl.d) (void)hipFree(sl.d);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    for (void *v : s->d_vec)
        if (v) (void)hipFree(v);
    for (auto &r : s->ev_pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    delete s;
    return QSV_OK;
}

qsv_status qsv_allocate(qsv_sim *s, int32_t count, int32_t *ids_out) {
    QSV_CHECK(s);
    if (count < 0) return fail(s, QSV_EINVAL, "count must be >= 0");
    if (s->n + count > s->opt.n_max)
        return fail(s, QSV_ENOMEM, "allocation exceeds n_max = " + std::to_string(s->opt.n_max));
    if (count == 0) return QSV_OK;
    const int n_new = s->n + count;
    if (s->materialized) {
        QSV_TRY(ensure_capacity(s, n_new));
        QSV_HIP(s, qsv::dev::zero_range(s->opt.dtype, s->d_state, 1ull << s->n, 1ull << n_new,
                                        s->stream));
    }
    for (int c = 0; c < count; ++c) {
        int id = 0;
        while (s->pos_of[id] >= 0) ++id;
        s->pos_of[id] = s->n;
        s->id_at.push_back(id);
        s->n += 1;
        if (ids_out) ids_out[c] = id;
    }
    return QSV_OK;
}

qsv_status qsv_deallocate(qsv_sim *s, int32_t id) {
    QSV_CHECK(s);
    if (id < 0 || id >= 64 || s->pos_of[id] < 0)
        return fail(s, QSV_EINVAL, "unknown qubit id " + std::to_string(id));
    const int pos = s->pos_of[id];
    if (s->materialized || !s->queue.empty()) {
        QSV_TRY(do_flush(s));
        double p0, p1;
        QSV_TRY(prob_split_host(s, pos, &p0, &p1));
        const double tau = s->opt.dtype == QSV_C128 ? 1e-12 : 1e-6;
        int value;
        if (p1 <= tau) value = 0;
        else if (p0 <= tau) value = 1;
        else
            return fail(s, QSV_ENOTCLASSICAL,
                        "qubit " + std::to_string(id) + " is in superposition (p1 = " +
                            std::to_string(p1) + ")");
        if (s->n == 1) {
            // the state becomes the 0-qubit state |> = 1; keep the amplitude's phase
            // by compacting into the first element
        }
        const uint64_t half = s->dim() >> 1;
        // compact into the upper part of a scratch vector, then copy back
        void *tmp = nullptr;
        QSV_HIP(s, hipMalloc(&tmp, std::max<uint64_t>(half, 1) * s->elem()));
        hipError_t e = qsv::dev::compact(s->opt.dtype, s->d_state, tmp, s->n, pos, value, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->d_state, tmp, half * s->elem(), hipMemcpyDeviceToDevice, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        (void)hipFree(tmp);
        if (e != hipSuccess) return hip_fail(s, e, "dealloc compaction");
        s->stats.kernels += 1;
        s->stats.alg_bytes += 2.0 * half * s->elem();
    }
    // bookkeeping: remove bit `pos`
    s->id_at.erase(s->id_at.begin() + pos);
    s->pos_of[id] = -1;
    for (int p = pos; p < (int)s->id_at.size(); ++p) s->pos_of[s->id_at[p]] = p;
    s->n -= 1;
    return QSV_OK;
}

qsv_status qsv_qubits(const qsv_sim *s, int32_t *n, int32_t *ids) {
    if (!live(s)) return fail(nullptr, QSV_ESTATE, "invalid or destroyed handle");
    if (n) *n = s->n;
    if (ids)
        for (int p = 0; p < s->n; ++p) ids[p] = s->id_at[p];
    return QSV_OK;
}

qsv_status qsv_apply(qsv_sim *s, const double *U, int32_t k, const int32_t *targets, int32_t c,
                     const int32_t *controls) {
    QSV_CHECK(s);
    if (!U || !targets || (c > 0 && !controls)) return fail(s, QSV_EINVAL, "NULL argument");
    if (k < 1 || k > qsv::kMaxK) return fail(s, QSV_EINVAL, "k must be in 1..5");
    if (c < 0 || c + k > s->n) return fail(s, QSV_EINVAL, "too many qubits for the register");
    Gate g;
    g.k = k;
    uint64_t seen = 0;
    for (int j = 0; j < k; ++j) {
        const int id = targets[j];
        if (id < 0 || id >= 64 || s->pos_of[id] < 0)
            return fail(s, QSV_EINVAL, "unknown target qubit id " + std::to_string(id));
        const int p = s->pos_of[id];
        if (seen & (1ull << p)) return fail(s, QSV_EINVAL, "qubit repeated in the gate");
        seen |= 1ull << p;
        g.t[j] = p;
    }
    for (int j = 0; j < c; ++j) {
        const int id = controls[j];
        if (id < 0 || id >= 64 || s->pos_of[id] < 0)
            return fail(s, QSV_EINVAL, "unknown control qubit id " + std::to_string(id));
        const int p = s->pos_of[id];
        if (seen & (1ull << p)) return fail(s, QSV_EINVAL, "qubit repeated in the gate");
        seen |= 1ull << p;
        g.ctrl |= 1ull << p;
    }
    const int D = 1 << k;
    g.U.resize((size_t)D * D);
    for (int i = 0; i < D * D; ++i) {
        const double re = U[2 * i], im = U[2 * i + 1];
        if (!std::isfinite(re) || !std::isfinite(im))
            return fail(s, QSV_EINVAL, "non-finite matrix entry");
        g.U[i] = cd(re, im);
    }
    s->queue.push_back(std::move(g));
    const int lim = s->opt.queue_limit > 0 ? s->opt.queue_limit : 4096;
    if ((int)s->queue.size() >= lim) return do_flush(s);
    return QSV_OK;
}

qsv_status qsv_apply_diag(qsv_sim *s, const double *d, int32_t k, const int32_t *targets,
                          int32_t c, const int32_t *controls) {
    QSV_CHECK(s);
    if (!d) return fail(s, QSV_EINVAL, "NULL diagonal");
    if (k < 1 || k > qsv::kMaxK) return fail(s, QSV_EINVAL, "k must be in 1..5");
    const int D = 1 << k;
    std::vector<double> U((size_t)D * D * 2, 0.0);
    for (int r = 0; r < D; ++r) {
        U[2 * ((size_t)r * D + r)] = d[2 * r];
        U[2 * ((size_t)r * D + r) + 1] = d[2 * r + 1];
    }
    return qsv_apply(s, U.data(), k, targets, c, controls);
}

qsv_status qsv_flush(qsv_sim *s) {
    QSV_CHECK(s);
    return do_flush(s);
}


qsv_status qsv_dm_apply(qsv_sim *s, const double *U, int32_t k, const int32_t *targets,
                        int32_t c, const int32_t *controls) {
    QSV_CHECK(s);
    if (!U) return fail(s, QSV_EINVAL, "NULL argument");
    uint64_t tm, cm;
    QSV_TRY(dm_check(s, k, targets, c, controls, 2, &tm, &cm));
    const int n = s->n / 2;
    const int D = 1 << k;
    Gate row, col;
    row.k = col.k = k;
    row.U.resize((size_t)D * D);
    col.U.resize((size_t)D * D);
    for (int i = 0; i < D * D; ++i) {
        const double re = U[2 * i], im = U[2 * i + 1];
        if (!std::isfinite(re) || !std::isfinite(im))
            return fail(s, QSV_EINVAL, "non-finite matrix entry");
        row.U[i] = cd(re, im);
        col.U[i] = cd(re, -im);
    }
    for (int j = 0; j < k; ++j) {
        row.t[j] = targets[j];
        col.t[j] = targets[j] + n;
    }
    row.ctrl = cm;
    col.ctrl = cm << n;
    dm_queue(s, std::move(row));
    dm_queue(s, std::move(col));
    const int lim = s->opt.queue_limit > 0 ? s->opt.queue_limit : 4096;
    if ((int)s->queue.size() >= lim) return do_flush(s);
    return QSV_OK;
}

qsv_status qsv_dm_apply_kraus(qsv_sim *s, int32_t nk, const double *kraus, int32_t k,
                              const int32_t *targets) {
    QSV_CHECK(s);
    if (!kraus || nk < 1) return fail(s, QSV_EINVAL, "no Kraus matrices");
    uint64_t tm, cm;
    QSV_TRY(dm_check(s, k, targets, 0, nullptr, 2, &tm, &cm));
    const int n = s->n / 2;
    const int D = 1 << k, DD = D * D;
    for (size_t i = 0; i < (size_t)2 * nk * D * D; ++i)
        if (!std::isfinite(kraus[i])) return fail(s, QSV_EINVAL, "non-finite Kraus entry");
    // local index of the 2k-qubit op: row bits r (targets) low, column bits c high
    Gate g;
    g.k = 2 * k;
    for (int j = 0; j < k; ++j) {
        g.t[j] = targets[j];
        g.t[k + j] = targets[j] + n;
    }
    g.U.assign((size_t)DD * DD, cd(0, 0));
    for (int j = 0; j < nk; ++j) {
        const double *K = kraus + (size_t)2 * j * D * D;
        auto kv = [&](int a, int b) { return cd(K[2 * (a * D + b)], K[2 * (a * D + b) + 1]); };
        for (int r2 = 0; r2 < D; ++r2)
            for (int c2 = 0; c2 < D; ++c2)
                for (int r = 0; r < D; ++r)
                    for (int c = 0; c < D; ++c)
                        g.U[(size_t)(r2 + D * c2) * DD + (r + D * c)] +=
                            kv(r2, r) * std::conj(kv(c2, c));
    }
    dm_queue(s, std::move(g));
    const int lim = s->opt.queue_limit > 0 ? s->opt.queue_limit : 4096;
    if ((int)s->queue.size() >= lim) return do_flush(s);
    return QSV_OK;
}

qsv_status qsv_dm_probabilities(qsv_sim *s, double *out) {
    QSV_CHECK(s);
    if (!out) return fail(s, QSV_EINVAL, "NULL argument");
    if ((s->n & 1) || s->n == 0)
        return fail(s, QSV_EINVAL, "a density matrix needs an even, nonzero number of qubits");
    const int n = s->n / 2;
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    QSV_TRY(ensure_ws(s, 8ull << n));
    QSV_HIP(s, qsv::dev::dm_diagonal(s->opt.dtype, s->d_state, n, (double *)s->d_ws, s->stream));
    QSV_HIP(s, hipMemcpyAsync(out, s->d_ws, 8ull << n, hipMemcpyDeviceToHost, s->stream));
    return sync(s);
}

qsv_status qsv_dm_expectation(qsv_sim *s, int32_t nterms, const uint64_t *xmask,
                              const uint64_t *zmask, const double *coeff, double *out) {
    QSV_CHECK(s);
    if (!out || nterms < 0 || (nterms > 0 && (!xmask || !zmask || !coeff)))
        return fail(s, QSV_EINVAL, "NULL argument");
    if ((s->n & 1) || s->n == 0)
        return fail(s, QSV_EINVAL, "a density matrix needs an even, nonzero number of qubits");
    const int n = s->n / 2;
    const uint64_t full = (1ull << n) - 1;
    for (int t = 0; t < nterms; ++t)
        if (((xmask[t] | zmask[t]) & ~full) || !std::isfinite(coeff[t]))
            return fail(s, QSV_EINVAL, "Pauli term outside the system qubits");
    *out = 0.0;
    if (nterms == 0) return QSV_OK;
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    const size_t off_z = 8 * (size_t)nterms, off_p = 16 * (size_t)nterms;
    QSV_TRY(ensure_ws(s, off_p + 16 * (size_t)nterms));
    unsigned char *w = (unsigned char *)s->d_ws;
    std::vector<unsigned char> meta(off_p);
    std::memcpy(meta.data(), xmask, 8 * (size_t)nterms);
    std::memcpy(meta.data() + off_z, zmask, 8 * (size_t)nterms);
    QSV_HIP(s, hipMemcpyAsync(w, meta.data(), off_p, hipMemcpyHostToDevice, s->stream));
    QSV_HIP(s, qsv::dev::dm_pauli_sums(s->opt.dtype, s->d_state, n, nterms, (const uint64_t *)w,
                                       (const uint64_t *)(w + off_z), (double *)(w + off_p),
                                       s->stream));
    std::vector<double> part(2 * (size_t)nterms);
    QSV_HIP(s, hipMemcpyAsync(part.data(), w + off_p, 16 * (size_t)nterms, hipMemcpyDeviceToHost,
                              s->stream));
    QSV_TRY(sync(s));
    // Tr(rho P) = i^ny * sum_r (-1)^popcount(r & z) rho[r][r ^ x]
    double acc = 0.0;
    for (int t = 0; t < nterms; ++t) {
        const int ny = popc(xmask[t] & zmask[t]) & 3;
        const double re = part[2 * t], im = part[2 * t + 1];
        const double tr = ny == 0 ? re : ny == 1 ? -im : ny == 2 ? -re : im;
        acc += coeff[t] * tr;
    }
    *out = acc;
    return QSV_OK;
}

qsv_status qsv_apply_math(qsv_sim *s, int32_t w, const int32_t *qubits, const uint32_t *table,
                          int32_t c, const int32_t *controls) {
    QSV_CHECK(s);
    if (!qubits || !table || (c > 0 && !controls)) return fail(s, QSV_EINVAL, "NULL argument");
    if (w < 1 || w > qsv::dev::kMaxMathBits)
        return fail(s, QSV_EINVAL, "register width must be in 1..26");
    if (c < 0 || w + c > s->n) return fail(s, QSV_EINVAL, "too many qubits for the register");
    uint64_t regmask = 0, ctrl = 0;
    QSV_TRY(check_ids(s, w, qubits, &regmask));
    QSV_TRY(check_ids(s, c, controls, &ctrl));
    if (regmask & ctrl) return fail(s, QSV_EINVAL, "a control is also a register qubit");
    // the table must be a bijection; the kernel gathers through its inverse
    const uint32_t size = 1u << w;
    std::vector<uint32_t> inv(size, 0xffffffffu);
    for (uint32_t x = 0; x < size; ++x) {
        const uint32_t y = table[x];
        if (y >= size || inv[y] != 0xffffffffu)
            return fail(s, QSV_EINVAL, "math table is not a permutation of 0..2^w-1");
        inv[y] = x;
    }
    qsv::dev::MathArgs a{};
    a.regmask = regmask;
    a.ctrl = ctrl;
    a.w = w;
    a.shift = s->pos_of[qubits[0]];
    for (int b = 0; b < w; ++b) {
        a.pos[b] = (uint32_t)s->pos_of[qubits[b]];
        if ((int)a.pos[b] != a.shift + b) a.shift = -1;
    }
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    if (s->alt_amps < s->cap_amps) {
        if (s->d_alt) {
            QSV_HIP(s, hipStreamSynchronize(s->stream));
            QSV_HIP(s, hipFree(s->d_alt));
            s->d_alt = nullptr;
            s->alt_amps = 0;
        }
        hipError_t e = hipMalloc(&s->d_alt, s->cap_amps * s->elem());
        if (e != hipSuccess) {
            (void)hipGetLastError();
            s->d_alt = nullptr;
            return fail(s, QSV_ENOMEM, "hipMalloc of the math gate's second state buffer failed");
        }
        s->alt_amps = s->cap_amps;
    }
    void *dinv = nullptr;
    QSV_TRY(stage(s, inv.data(), (size_t)size * sizeof(uint32_t), &dinv));
    const int tok = tbegin(s);
    QSV_HIP(s, qsv::dev::math_gather(s->opt.dtype, s->d_state, s->d_alt, s->dim(), a,
                                     (const uint32_t *)dinv, s->stream));
    tend(s, tok, QSV_K_MONO, 2.0 * (double)s->dim() * s->elem());
    if (s->owns_state) {
        std::swap(s->d_state, s->d_alt);
        std::swap(s->cap_amps, s->alt_amps);
    } else {
        QSV_HIP(s, hipMemcpyAsync(s->d_state, s->d_alt, s->dim() * s->elem(),
                                  hipMemcpyDeviceToDevice, s->stream));
    }
    s->stats.gates += 1;
    s->stats.amp_gate_updates += (double)s->dim();
    return QSV_OK;
}

qsv_status qsv_synchronize(qsv_sim *s) {
    QSV_CHECK(s);
    if (!s->materialized) return QSV_OK;
    return sync(s);
}

qsv_status qsv_get_probability(qsv_sim *s, int32_t m, const int32_t *qubits, const int8_t *bits,
                               double *out) {
    QSV_CHECK(s);
    if (!out || m < 0 || (m > 0 && (!qubits || !bits))) return fail(s, QSV_EINVAL, "bad argument");
    uint64_t mask;
    QSV_TRY(check_ids(s, m, qubits, &mask));
    uint64_t ones = 0;
    for (int j = 0; j < m; ++j)
        if (bits[j]) ones |= 1ull << s->pos_of[qubits[j]];
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    QSV_TRY(ensure_ws(s, qsv::dev::reduce_workspace_bytes(s->n)));
    qsv::dev::IndexArgs ia;
    index_args(mask, ones, ia);
    const int tok = tbegin(s);
    QSV_HIP(s, qsv::dev::prob_masked(s->opt.dtype, s->d_state, 1ull << (s->n - m), ia,
                                     (double *)s->d_ws, s->d_small, s->stream));
    tend(s, tok, QSV_K_REDUCE, (double)(1ull << (s->n - m)) * s->elem());
    QSV_HIP(s, hipMemcpyAsync(out, s->d_small, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    s->stats.kernels += 2;
    s->stats.alg_bytes += (double)(1ull << (s->n - m)) * s->elem();
    return sync(s);
}

qsv_status qsv_get_probability_noalloc(const void *state, int32_t dtype, int32_t n, int32_t m,
                                       const int32_t *positions, const int8_t *bits,
                                       double *out_dev, void *stream) {
    if (!state || !out_dev) return fail(nullptr, QSV_EINVAL, "NULL state or output");
    if (dtype != QSV_C128 && dtype != QSV_C64) return fail(nullptr, QSV_EINVAL, "bad dtype");
    if (n < 0 || n > qsv::kMaxQubits) return fail(nullptr, QSV_EINVAL, "n outside 0..36");
    if (m < 0 || m > n || (m > 0 && (!positions || !bits)))
        return fail(nullptr, QSV_EINVAL, "bad mask (m outside 0..n or NULL arrays)");
    uint64_t mask = 0, ones = 0;
    for (int j = 0; j < m; ++j) {
        const int p = positions[j];
        if (p < 0 || p >= n || ((mask >> p) & 1))
            return fail(nullptr, QSV_EINVAL, "position outside 0..n-1 or repeated");
        mask |= 1ull << p;
        if (bits[j]) ones |= 1ull << p;
    }
    const uint64_t ngroups = 1ull << (n - m);
    if (qsv::dev::prob_noalloc_partials(ngroups) > qsv::dev::prob_noalloc_capacity())
        return fail(nullptr, QSV_EINVAL, "partial sums exceed the static scratch array");
    qsv::dev::IndexArgs ia;
    index_args(mask, ones, ia);
    const hipError_t e = qsv::dev::prob_masked_noalloc(dtype, state, ngroups, ia, out_dev,
                                                       (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(nullptr, QSV_EDEVICE, std::string("qsv_get_probability_noalloc: ") + hipGetErrorString(e));
    return QSV_OK;
}

qsv_status qsv_get_probabilities(qsv_sim *s, double *out, int32_t out_is_device) {
    QSV_CHECK(s);
    if (!out) return fail(s, QSV_EINVAL, "NULL output");
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    s->stats.kernels += 1;
    s->stats.alg_bytes += (double)s->dim() * (s->elem() + 8);
    if (out_is_device) {
        QSV_HIP(s, qsv::dev::probs(s->opt.dtype, s->d_state, s->dim(), out, s->stream));
        return sync(s);
    }
    QSV_TRY(ensure_ws(s, s->dim() * sizeof(double)));
    QSV_HIP(s, qsv::dev::probs(s->opt.dtype, s->d_state, s->dim(), (double *)s->d_ws, s->stream));
    QSV_HIP(s, hipMemcpyAsync(out, s->d_ws, s->dim() * sizeof(double), hipMemcpyDeviceToHost,
                              s->stream));
    return sync(s);
}

// Pauli sum over bit positions (shared by the ABI call and the adjoint).
static qsv_status expectation_positions(qsv_sim *s, const void *psi, int nq, int nterms,
                                        const uint64_t *x, const uint64_t *z, const double *c,
                                        double *re_out, double *im_out) {
    std::vector<int> order(nterms);
    for (int t = 0; t < nterms; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return x[a] < x[b]; });
    std::vector<uint64_t> zs(nterms + 1);
    std::vector<double> cs(nterms + 1);
    std::vector<int32_t> ny(nterms + 1);
    std::vector<qsv::dev::PauliGroup> groups;
    for (int i = 0; i < nterms; ++i) {
        const int t = order[i];
        zs[i] = z[t];
        cs[i] = c[t];
        ny[i] = popc(x[t] & z[t]);
        if (groups.empty() || groups.back().x != x[t]) groups.push_back({x[t], i, 0});
        groups.back().count += 1;
    }
    int nchunks = 0;
    for (auto &g : groups) nchunks += (g.count + 7) / 8;
    const size_t meta = ((nterms + 1) * (8 + 8 + 4) + 255) & ~size_t(255);
    const size_t need = qsv::dev::pauli_workspace_bytes(nq, nchunks, nterms) + meta + 4096;
    QSV_TRY(ensure_ws(s, need));
    unsigned char *w = (unsigned char *)s->d_ws;
    uint64_t *dz = (uint64_t *)w;
    double *dc = (double *)(w + 8 * (nterms + 1));
    int32_t *dny = (int32_t *)(w + 16 * (nterms + 1));
    std::vector<unsigned char> hostmeta(meta, 0);
    std::memcpy(hostmeta.data(), zs.data(), 8 * (nterms + 1));
    std::memcpy(hostmeta.data() + 8 * (nterms + 1), cs.data(), 8 * (nterms + 1));
    std::memcpy(hostmeta.data() + 16 * (nterms + 1), ny.data(), 4 * (nterms + 1));
    QSV_HIP(s, hipMemcpyAsync(w, hostmeta.data(), meta, hipMemcpyHostToDevice, s->stream));
    QSV_HIP(s, hipStreamSynchronize(s->stream));
    double *ws = (double *)(w + meta);
    const int tok = tbegin(s);
    QSV_HIP(s, qsv::dev::pauli_expectation(s->opt.dtype, psi, nq, (int)groups.size(), groups.data(),
                                           dz, dc, dny, nterms, ws, s->ws_bytes - meta,
                                           s->d_small, s->stream, zs.data()));
    tend(s, tok, QSV_K_REDUCE, (double)nchunks * (double)(1ull << nq) * s->elem());
    double h[2];
    QSV_HIP(s, hipMemcpyAsync(h, s->d_small, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    QSV_TRY(sync(s));
    s->stats.kernels += 2;
    s->stats.alg_bytes += (double)nchunks * (double)(1ull << nq) * s->elem();
    *re_out = h[0];
    if (im_out) *im_out = h[1];
    return QSV_OK;
}

qsv_status qsv_get_expectation_complex(qsv_sim *s, int32_t nterms, const uint64_t *xmask,
                                       const uint64_t *zmask, const double *coeff, double *re_out,
                                       double *im_out) {
    QSV_CHECK(s);
    if (!re_out || !im_out || nterms < 0 || (nterms > 0 && (!xmask || !zmask || !coeff)))
        return fail(s, QSV_EINVAL, "bad argument");
    std::vector<uint64_t> x(nterms), z(nterms);
    for (int t = 0; t < nterms; ++t) {
        uint64_t xm = 0, zm = 0;
        for (int id = 0; id < 64; ++id) {
            const bool bx = (xmask[t] >> id) & 1, bz = (zmask[t] >> id) & 1;
            if (!bx && !bz) continue;
            if (s->pos_of[id] < 0)
                return fail(s, QSV_EINVAL, "Pauli term on unknown qubit id " + std::to_string(id));
            if (bx) xm |= 1ull << s->pos_of[id];
            if (bz) zm |= 1ull << s->pos_of[id];
        }
        x[t] = xm;
        z[t] = zm;
    }
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    return expectation_positions(s, s->d_state, s->n, nterms, x.data(), z.data(), coeff, re_out,
                                 im_out);
}

qsv_status qsv_get_expectation(qsv_sim *s, int32_t nterms, const uint64_t *xmask,
                               const uint64_t *zmask, const double *coeff, double *out) {
    QSV_CHECK(s);
    if (!out) return fail(s, QSV_EINVAL, "bad argument");
    double im = 0.0;
    return qsv_get_expectation_complex(s, nterms, xmask, zmask, coeff, out, &im);
}

qsv_status qsv_measure(qsv_sim *s, int32_t m, const int32_t *qubits, const double *u,
                       int8_t *bits_out) {
    QSV_CHECK(s);
    if (m < 0 || (m > 0 && (!qubits || !u || !bits_out))) return fail(s, QSV_EINVAL, "bad argument");
    QSV_TRY(check_ids(s, m, qubits, nullptr));
    for (int j = 0; j < m; ++j)
        if (!(u[j] >= 0.0 && u[j] < 1.0)) return fail(s, QSV_EINVAL, "uniform outside [0,1)");
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    for (int j = 0; j < m; ++j) {
        const int pos = s->pos_of[qubits[j]];
        double p0, p1;
        QSV_TRY(prob_split_host(s, pos, &p0, &p1));
        const int outcome = (u[j] * (p0 + p1) < p0) ? 0 : 1;
        const double keep = outcome ? p1 : p0;
        if (!(keep > 0.0)) return fail(s, QSV_EDEVICE, "measured branch has zero probability");
        QSV_HIP(s, qsv::dev::collapse(s->opt.dtype, s->d_state, s->n, pos, outcome,
                                      1.0 / std::sqrt(keep), s->stream));
        s->stats.kernels += 1;
        s->stats.alg_bytes += 2.0 * s->dim() * s->elem();
        bits_out[j] = (int8_t)outcome;
    }
    return sync(s);
}

qsv_status qsv_apply_kraus_sampled(qsv_sim *s, int32_t nk, const double *kraus, int32_t k,
                                   const int32_t *targets, double u, int32_t *chosen,
                                   double *probs) {
    QSV_CHECK(s);
    if (nk < 1 || !kraus || !targets || !chosen) return fail(s, QSV_EINVAL, "bad argument");
    if (k < 1 || k > 2) return fail(s, QSV_EINVAL, "k must be 1 or 2");
    if (!(u >= 0.0 && u < 1.0)) return fail(s, QSV_EINVAL, "uniform outside [0,1)");
    QSV_TRY(check_ids(s, k, targets, nullptr));
    const int D = 1 << k;
    for (int i = 0; i < nk * D * D * 2; ++i)
        if (!std::isfinite(kraus[i])) return fail(s, QSV_EINVAL, "non-finite Kraus entry");
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    // reduced density matrix of the targets (bit j of its index = target j)
    int pos[2] = {s->pos_of[targets[0]], k > 1 ? s->pos_of[targets[1]] : 0};
    QSV_TRY(ensure_ws(s, qsv::dev::reduced_dm_workspace_bytes()));
    const int tok = tbegin(s);
    QSV_HIP(s, qsv::dev::reduced_dm(s->opt.dtype, s->d_state, s->n, k, pos, (double *)s->d_ws,
                                    s->d_small, s->stream));
    tend(s, tok, QSV_K_REDUCE, (double)s->dim() * s->elem());
    double h[32];
    QSV_HIP(s, hipMemcpyAsync(h, s->d_small, sizeof(double) * 2 * D * D, hipMemcpyDeviceToHost,
                              s->stream));
    s->stats.kernels += 2;
    s->stats.alg_bytes += (double)s->dim() * s->elem();
    QSV_TRY(sync(s));
    std::vector<cd> rho((size_t)D * D);
    for (int e = 0; e < D * D; ++e) rho[e] = cd(h[2 * e], h[2 * e + 1]);
    // p_j = ||K_j psi||^2 = Tr(K_j rho K_j^dagger)
    std::vector<double> p(nk);
    double total = 0.0;
    for (int j = 0; j < nk; ++j) {
        const double *K = kraus + (size_t)j * D * D * 2;
        double pj = 0.0;
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b)
                for (int c = 0; c < D; ++c) {
                    const cd kab(K[2 * (a * D + b)], K[2 * (a * D + b) + 1]);
                    const cd kac(K[2 * (a * D + c)], K[2 * (a * D + c) + 1]);
                    pj += (kab * rho[b * D + c] * std::conj(kac)).real();
                }
        p[j] = std::max(pj, 0.0);
        total += p[j];
    }
    if (probs)
        for (int j = 0; j < nk; ++j) probs[j] = p[j];
    if (!(total > 0.0) || !std::isfinite(total))
        return fail(s, QSV_EINVAL, "the channel leaves no probability");
    // the first branch whose running sum exceeds u * total
    const double r = u * total;
    int pick = -1;
    double run = 0.0;
    for (int j = 0; j < nk; ++j) {
        run += p[j];
        if (run > r) {
            pick = j;
            break;
        }
    }
    if (pick < 0)
        for (int j = nk - 1; j >= 0 && pick < 0; --j)
            if (p[j] > 0.0) pick = j;
    *chosen = pick;
    // queue K_pick / sqrt(p_pick): the state keeps unit norm
    const double sc = 1.0 / std::sqrt(p[pick]);
    std::vector<double> G((size_t)D * D * 2);
    for (int i = 0; i < D * D * 2; ++i) G[i] = kraus[(size_t)pick * D * D * 2 + i] * sc;
    return qsv_apply(s, G.data(), k, targets, 0, nullptr);
}

qsv_status qsv_sample(qsv_sim *s, int32_t shots, const double *u, uint64_t *out) {
    QSV_CHECK(s);
    if (shots < 0 || (shots > 0 && (!u || !out))) return fail(s, QSV_EINVAL, "bad argument");
    for (int j = 0; j < shots; ++j)
        if (!(u[j] >= 0.0 && u[j] < 1.0)) return fail(s, QSV_EINVAL, "uniform outside [0,1)");
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    if (shots == 0) return QSV_OK;
    const size_t wsb = qsv::dev::sample_workspace_bytes(s->n);
    const size_t ub = ((size_t)shots * 8 + 255) & ~size_t(255);
    QSV_TRY(ensure_ws(s, wsb + 2 * ub + 256));
    unsigned char *w = (unsigned char *)s->d_ws;
    double *du = (double *)w;
    uint64_t *dout = (uint64_t *)(w + ub);
    double *dws = (double *)(w + 2 * ub);
    QSV_HIP(s, hipMemcpyAsync(du, u, shots * sizeof(double), hipMemcpyHostToDevice, s->stream));
    const int tok = tbegin(s);
    QSV_HIP(s, qsv::dev::sample(s->opt.dtype, s->d_state, s->n, shots, du, dws, dout, s->stream));
    tend(s, tok, QSV_K_REDUCE, (double)s->dim() * s->elem());
    QSV_HIP(s, hipMemcpyAsync(out, dout, shots * sizeof(uint64_t), hipMemcpyDeviceToHost, s->stream));
    s->stats.kernels += 3;
    s->stats.alg_bytes += (double)s->dim() * s->elem();
    return sync(s);
}

qsv_status qsv_get_state(qsv_sim *s, void *dst, int32_t dst_is_device) {
    QSV_CHECK(s);
    if (!dst) return fail(s, QSV_EINVAL, "NULL destination");
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    QSV_HIP(s, hipMemcpyAsync(dst, s->d_state, s->dim() * s->elem(),
                              dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                              s->stream));
    return sync(s);
}

qsv_status qsv_set_state(qsv_sim *s, const void *src, int32_t src_is_device) {
    QSV_CHECK(s);
    if (!src) return fail(s, QSV_EINVAL, "NULL source");
    s->queue.clear();
    s->invalid = false;
    QSV_TRY(ensure_capacity(s, s->n));
    if (!s->d_small) QSV_HIP(s, hipMalloc((void **)&s->d_small, 64 * sizeof(double)));
    QSV_HIP(s, hipMemcpyAsync(s->d_state, src, s->dim() * s->elem(),
                              src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              s->stream));
    s->materialized = true;
    return sync(s);
}

qsv_status qsv_get_amplitudes(qsv_sim *s, int64_t count, const uint64_t *indices, double *out) {
    QSV_CHECK(s);
    if (count < 0 || (count > 0 && (!indices || !out))) return fail(s, QSV_EINVAL, "bad argument");
    for (int64_t i = 0; i < count; ++i)
        if (indices[i] >= (1ull << s->n)) return fail(s, QSV_EINVAL, "amplitude index out of range");
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    if (count == 0) return QSV_OK;
    const size_t ib = ((size_t)count * 8 + 255) & ~size_t(255);
    QSV_TRY(ensure_ws(s, ib + (size_t)count * 16));
    uint64_t *di = (uint64_t *)s->d_ws;
    double *dout = (double *)((unsigned char *)s->d_ws + ib);
    QSV_HIP(s, hipMemcpyAsync(di, indices, count * 8, hipMemcpyHostToDevice, s->stream));
    QSV_HIP(s, qsv::dev::gather(s->opt.dtype, s->d_state, di, (uint64_t)count, dout, s->stream));
    QSV_HIP(s, hipMemcpyAsync(out, dout, count * 16, hipMemcpyDeviceToHost, s->stream));
    return sync(s);
}

qsv_status qsv_state_pointer(qsv_sim *s, void **ptr, void **stream) {
    QSV_CHECK(s);
    QSV_TRY(do_flush(s));
    QSV_TRY(materialize(s));
    if (ptr) *ptr = s->d_state;
    if (stream) *stream = (void *)s->stream;
    return QSV_OK;
}

qsv_status qsv_get_stats(const qsv_sim *s, qsv_stats *out) {
    if (!live(s)) return fail(nullptr, QSV_ESTATE, "invalid or destroyed handle");
    if (!out) return QSV_EINVAL;
    *out = s->stats;
    return QSV_OK;
}

qsv_status qsv_reset_stats(qsv_sim *s) {
    QSV_CHECK(s);
    s->stats = qsv_stats{};
    QSV_TRY(collect_times(s));
    for (int c = 0; c < QSV_K_COUNT; ++c) {
        s->k_ms[c] = 0.0;
        s->k_launch[c] = 0;
        s->k_bytes[c] = 0.0;
    }
    return QSV_OK;
}

qsv_status qsv_get_kernel_times(qsv_sim *s, int32_t kclass, double *ms, uint64_t *launches,
                                double *alg_bytes) {
    QSV_CHECK(s);
    if (kclass < 0 || kclass >= QSV_K_COUNT) return fail(s, QSV_EINVAL, "unknown kernel class");
    QSV_TRY(collect_times(s));
    if (ms) *ms = s->k_ms[kclass];
    if (launches) *launches = s->k_launch[kclass];
    if (alg_bytes) *alg_bytes = s->k_bytes[kclass];
    return QSV_OK;
}

qsv_status qsv_reset(qsv_sim *s) {
    QSV_CHECK(s);
    s->queue.clear();
    s->invalid = false;
    if (!s->materialized) return QSV_OK;
    QSV_HIP(s, qsv::dev::fill_basis0(s->opt.dtype, s->d_state, s->dim(), s->stream));
    return QSV_OK;
}

qsv_status qsv_check_tile_programs(qsv_sim *s, double *state, int32_t *info) {
    QSV_CHECK(s);
    if (s->opt.mode != QSV_MODE_TILED) return fail(s, QSV_EINVAL, "handle is not in tiled mode");
    std::vector<Op> ops = canonical_queue(s, nullptr);
    const int m = std::min(tile_bits_for(s), s->n);
    std::vector<Pass> passes = plan_flush(s, ops, m);
    const int rb = reg_bits_for(s);
    std::vector<cd> psi(state ? s->dim() : 0);
    for (uint64_t i = 0; state && i < s->dim(); ++i) psi[i] = cd(state[2 * i], state[2 * i + 1]);
    int32_t counts[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (const Pass &ps : passes) {
        std::vector<double> mats;
        qsv::TileProgram pg;
        qsv::compile_pass(ps, rb, mats, pg, (int)s->elem());
        counts[0] += 1;
        if (!pg.reg) {
            char msg[160];
            std::snprintf(msg, sizeof msg,
                          "pass %d (tile %#llx, %d bits, %d register bits) runs on the LDS-tile kernel",
                          counts[0] - 1, (unsigned long long)ps.tile, pg.m, rb);
            if (log_level() >= 2)
                for (const Op &o : ps.ops)
                    std::fprintf(stderr, "  op kind=%d diag=%d k=%d t0=%d t1=%d ctrl=%#llx touch=%#x\n",
                                 o.kind, (int)o.diag, o.k, o.t[0], o.k > 1 ? o.t[1] : -1,
                                 (unsigned long long)o.ctrl, o.touch);
            return fail(s, QSV_EUNSUPPORTED, msg);
        }
        counts[1] += 1;
        counts[2] += pg.real_ops;
        counts[3] += pg.diag_ops;
        counts[4] += pg.remaps;
        counts[5] = std::max<int32_t>(counts[5], (int32_t)pg.img.size());
        counts[6] += (int32_t)pg.rops.size();
        counts[7] += pg.diag_merged;
        counts[8] += pg.local_remaps;
        counts[9] += pg.permutes ? 1 : 0;
        if (log_level() >= 2)
            std::fprintf(stderr, "qsv: check pass %d ops=%zu real=%d diag=%d remaps=%d rops=%zu image=%zuB\n",
                         counts[0] - 1, ps.ops.size(), pg.real_ops, pg.diag_ops, pg.remaps,
                         pg.rops.size(), pg.img.size());
        if (log_level() >= 3) {
            auto pos = [](uint64_t g) { return g ? __builtin_ctzll(g) : -1; };
            std::fprintf(stderr, "pass %d: load lanes", counts[0] - 1);
            for (int t = 0; t < 6; ++t) std::fprintf(stderr, " %d", pos(pg.g_thr[t]));
            std::fprintf(stderr, " | store lanes");
            for (int t = 0; t < 6; ++t) std::fprintf(stderr, " %d", pos(pg.g_thr_f[t]));
            std::fprintf(stderr, " | regs");
            for (int j = 0; j < rb; ++j) std::fprintf(stderr, " %d", pos(pg.g_reg[j]));
            std::fprintf(stderr, " -> ");
            for (int j = 0; j < rb; ++j) std::fprintf(stderr, " %d", pos(pg.g_reg_f[j]));
            std::fprintf(stderr, "\n");
        }
        if (!state) continue;
        const std::string err = qsv::emulate_reg_pass(pg, rb, mats, (int)s->elem(), s->n, psi);
        if (!err.empty()) return fail(s, QSV_EINVAL, "tile program check: " + err);
    }
    for (uint64_t i = 0; state && i < s->dim(); ++i) {
        state[2 * i] = psi[i].real();
        state[2 * i + 1] = psi[i].imag();
    }
    if (info) std::memcpy(info, counts, sizeof(counts));
    return QSV_OK;
}

qsv_status qsv_plan(qsv_sim *s, int32_t *n_ops, int32_t *n_passes, int32_t max_ops, int32_t *ks,
                    int32_t *targets, uint64_t *ctrls, double *mats) {
    QSV_CHECK(s);
    if (max_ops > 0 && (!ks || !targets || !ctrls || !mats)) return fail(s, QSV_EINVAL, "NULL output");
    std::vector<Op> ops = canonical_queue(s, nullptr);
    std::vector<Op> flat;
    int np = 0;
    if (s->opt.mode == QSV_MODE_PERGATE) {
        flat = ops;
        np = (int)ops.size();
    } else if (s->opt.mode == QSV_MODE_FUSED) {
        flat = qsv::fuse(ops, s->opt.k_max);
        np = (int)flat.size();
    } else {
        const int m = std::min(tile_bits_for(s), s->n);
        std::vector<Pass> passes = plan_flush(s, ops, m);
        np = (int)passes.size();
        flat = qsv::pass_ops_in_qubit_order(passes, s->n);
    }
    if (n_ops) *n_ops = (int32_t)flat.size();
    if (n_passes) *n_passes = np;
    for (int i = 0; i < (int)flat.size() && i < max_ops; ++i) {
        const Op &o = flat[i];
        ks[i] = o.k;
        for (int j = 0; j < 5; ++j) targets[5 * i + j] = j < o.k ? o.t[j] : -1;
        ctrls[i] = o.ctrl;
        std::vector<cd> U = qsv::dense_matrix(o);
        for (size_t e = 0; e < U.size(); ++e) {
            mats[(size_t)i * 2048 + 2 * e] = U[e].real();
            mats[(size_t)i * 2048 + 2 * e + 1] = U[e].imag();
        }
    }
    return QSV_OK;
}

}  // extern "C"

// ======================================================== adjoint gradient
namespace {

// Points the handle's launch machinery at another vector for a while.
struct StateSwap {
    qsv_sim *s;
    void *ptr;
    int n;
    StateSwap(qsv_sim *sim, void *buf, int nq) : s(sim), ptr(sim->d_state), n(sim->n) {
        s->d_state = buf;
        s->n = nq;
    }
    void to(void *buf) { s->d_state = buf; }
    ~StateSwap() {
        s->d_state = ptr;
        s->n = n;
    }
};

void rotation_matrix(int op, double theta, std::vector<cd> &U) {
    const double c = std::cos(theta / 2), sn = std::sin(theta / 2);
    if (op == QSV_OP_RX) U = {cd(c, 0), cd(0, -sn), cd(0, -sn), cd(c, 0)};
    else if (op == QSV_OP_RY) U = {cd(c, 0), cd(-sn, 0), cd(sn, 0), cd(c, 0)};
    else U = {std::polar(1.0, -theta / 2), cd(0, 0), cd(0, 0), std::polar(1.0, theta / 2)};
}

// Read gate g of a flat circuit (positions = circuit qubits).
qsv_status circuit_gate(qsv_sim *s, const qsv_circuit *c, int g, Gate &out, int *axis,
                        int *param) {
    const int k = c->k[g], nc = c->c[g], op = c->op[g];
    if (k < 1 || k > qsv::kMaxK || nc < 0 || k + nc > 8 || k + nc > c->n_qubits)
        return fail(s, QSV_EINVAL, "gate " + std::to_string(g) + ": bad qubit counts");
    out = Gate();
    out.k = k;
    uint64_t seen = 0;
    for (int j = 0; j < k + nc; ++j) {
        const int q = c->qubits[8 * g + j];
        if (q < 0 || q >= c->n_qubits || ((seen >> q) & 1))
            return fail(s, QSV_EINVAL, "gate " + std::to_string(g) + ": bad or repeated qubit");
        seen |= 1ull << q;
        if (j < k) out.t[j] = q;
        else out.ctrl |= 1ull << q;
    }
    *axis = 0;
    *param = -1;
    if (op == QSV_OP_MATRIX) {
        if (!c->matrices || !c->mat_off) return fail(s, QSV_EINVAL, "matrix gate without matrices");
        const int D = 1 << k;
        const double *m = c->matrices + 2 * c->mat_off[g];
        out.U.resize((size_t)D * D);
        for (int e = 0; e < D * D; ++e) {
            if (!std::isfinite(m[2 * e]) || !std::isfinite(m[2 * e + 1]))
                return fail(s, QSV_EINVAL, "non-finite matrix entry");
            out.U[e] = cd(m[2 * e], m[2 * e + 1]);
        }
    } else if (op >= QSV_OP_RX && op <= QSV_OP_RZ) {
        if (k != 1) return fail(s, QSV_EINVAL, "rotation gates act on one target");
        const int p = c->param ? c->param[g] : -1;
        if (p < 0 || p >= c->n_params || !c->params)
            return fail(s, QSV_EINVAL, "rotation gate " + std::to_string(g) + ": bad parameter index");
        const double th = c->params[p];
        if (!std::isfinite(th)) return fail(s, QSV_EINVAL, "non-finite angle");
        rotation_matrix(op, th, out.U);
        *axis = op;   // 1 = X, 2 = Y, 3 = Z
        *param = p;
    } else {
        return fail(s, QSV_EINVAL, "unknown gate op");
    }
    return QSV_OK;
}

qsv_status ensure_vectors(qsv_sim *s, uint64_t amps) {
    if (s->vec_amps >= amps && s->vec_dtype == s->opt.dtype) return QSV_OK;
    QSV_HIP(s, hipStreamSynchronize(s->stream));
    for (void *&v : s->d_vec)
        if (v) {
            QSV_HIP(s, hipFree(v));
            v = nullptr;
        }
    for (int i = 0; i < 2; ++i) {
        hipError_t e = hipMalloc(&s->d_vec[i], amps * s->elem());
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(s, QSV_ENOMEM, "hipMalloc of the adjoint vectors failed");
        }
    }
    s->vec_amps = amps;
    s->vec_dtype = s->opt.dtype;
    return QSV_OK;
}

qsv_status run_ops(qsv_sim *s, const std::vector<Op> &ops) {
    if (s->opt.mode == QSV_MODE_PERGATE) {
        for (const Op &op : ops) QSV_TRY(launch_op(s, op));
        return QSV_OK;
    }
    if (s->opt.mode == QSV_MODE_FUSED) {
        for (const Op &op : qsv::fuse(ops, s->opt.k_max)) QSV_TRY(launch_op(s, op));
        return QSV_OK;
    }
    const int m = std::min(tile_bits_for(s), s->n);
    return run_tile_passes(s, plan_flush(s, ops, m));
}

// Tile bits of the tiled reverse sweep: two tiles (psi, phi) per workgroup,
// sized so that two workgroups share a compute unit's LDS by default.
int adjoint_tile_bits(const qsv_sim *s, int n) {
    const int mmax = s->opt.dtype == QSV_C128 ? 12 : 13;
    int m = s->opt.tile_bits > 0 ? s->opt.tile_bits : (s->opt.dtype == QSV_C128 ? 11 : 12);
    return std::max(1, std::min({m, mmax, n}));
}

// The reverse sweep as LDS tile passes.  Steps are U_g^dagger in reverse
// gate order; rotation g keeps its slot (its index in reverse order) for the
// partial sums.  Steps move across each other only where the planner's
// commutation test allows; a rotation's generator commutes with everything
// its gate commutes with (diagonal on shared qubits, or disjoint), so moving
// steps leaves every recorded inner product unchanged.  Rotations that follow
// each other in a pass on the same target with the same controls become one
// chain step (up to kAdjChain), so their pairs pass through LDS once.
qsv_status adjoint_reverse_tiled(qsv_sim *s, const std::vector<Gate> &gates,
                                 const std::vector<int> &axis, const double *params,
                                 const std::vector<int> &param, void *psi, void *phi,
                                 double *partial, int grid, int mfma_k) {
    using qsv::dev::AdjOp;
    const int n = s->n;
    const int m = adjoint_tile_bits(s, n);
    std::vector<Op> steps;
    std::vector<int> saxis, sslot;
    std::vector<double> stheta;
    std::vector<qsv::PlanItem> items;
    int slot = 0;
    for (int g = (int)gates.size() - 1; g >= 0; --g) {
        const Gate &gt = gates[g];
        Op op;
        qsv::PlanItem it;
        if (axis[g]) {
            // addressing only: a dense one-target op on the gate's qubits
            op.kind = Op::DENSE;
            op.k = 1;
            op.t[0] = gt.t[0];
            op.ctrl = gt.ctrl;
            op.U = gt.U;
            it.need = 1ull << gt.t[0];
            it.mix = axis[g] == QSV_OP_RZ ? 0 : it.need;
            it.all = it.need | gt.ctrl;
            sslot.push_back(slot++);
            stheta.push_back(params[param[g]]);
        } else {
            const int D = 1 << gt.k;
            Gate d = gt;
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c)
                    d.U[(size_t)r * D + c] = std::conj(gt.U[(size_t)c * D + r]);
            if (!qsv::canonicalize(d, op)) continue;
            it.need = it.mix = op.mixing();
            it.all = op.qubits();
            sslot.push_back(-1);
            stheta.push_back(0.0);
        }
        saxis.push_back(axis[g]);
        steps.push_back(std::move(op));
        items.push_back(it);
    }
    const std::vector<qsv::PlanGroup> groups = qsv::plan_groups(items, n, m, 3);
    struct Launch {
        int group;
        size_t first, count;
        int nrot;
    };
    // a step waiting in the open block
    struct Pending {
        int i;            // step index
        uint32_t lctrl;   // in-tile controls (tile bits)
        uint64_t ectrl;   // controls outside the tile
        int kind;         // AdjSubKind
        int lslot;
    };
    const int eb = (int)s->elem();
    std::vector<double> mats;
    std::vector<AdjOp> aops;
    std::vector<qsv::dev::AdjSub> subs;
    std::vector<Launch> launches;
    auto push_c = [&](const cd &v) {
        mats.push_back(v.real());
        mats.push_back(v.imag());
    };
    for (int gi = 0; gi < (int)groups.size(); ++gi) {
        const uint64_t tile = groups[gi].tile;
        const int mt = popc(tile);
        int li[64];
        int c = 0;
        for (int p = 0; p < 64; ++p) li[p] = ((tile >> p) & 1) ? c++ : -1;
        // blocks of three tile bits take the one-target and diagonal steps
        const bool use_blocks = mt >= 3;
        Launch L{gi, aops.size(), 0, 0};
        int prev = -1;   // step index of the launch's last op if it is a chain
        bool bopen = false;
        uint32_t bbits = 0;
        std::vector<Pending> bq;
        auto close_block = [&]() {
            if (!bopen) return;
            for (int b = 0; b < mt && popc(bbits) < 3; ++b) bbits |= 1u << b;
            int bl[3], nb3 = 0;
            for (int b = 0; b < mt; ++b)
                if ((bbits >> b) & 1) bl[nb3++] = b;
            auto jpos = [&](int lb) { return lb == bl[0] ? 0 : lb == bl[1] ? 1 : 2; };
            auto bmask = [&](uint32_t lm) {
                int cm = 0;
                for (int j = 0; j < 3; ++j)
                    if ((lm >> bl[j]) & 1) cm |= 1 << j;
                return cm;
            };
            AdjOp a{};
            a.kind = qsv::dev::ADJ_BLOCK;
            qsv::dev::TileOp &t = a.op;
            t.k = 3;
            for (int r = 0; r < 8; ++r) {
                uint32_t o = 0;
                for (int j = 0; j < 3; ++j)
                    if ((r >> j) & 1) o |= 1u << bl[j];
                t.sl[r] = qsv::swz_elem(o, eb) * eb;
            }
            for (int b = 0; b < mt; ++b)
                if (!((bbits >> b) & 1)) t.fz[t.nfree++] = qsv::swz_elem(1u << b, eb) * eb;
            a.sub0 = (int32_t)subs.size();
            a.nsub = (int32_t)bq.size();
            for (const Pending &pq : bq) {
                const Op &st = steps[pq.i];
                qsv::dev::AdjSub u{};
                u.kind = pq.kind;
                u.ectrl = pq.ectrl;
                u.cmask = bmask(pq.lctrl);
                if (pq.kind == qsv::dev::SUB_ROT) {
                    u.j = jpos(li[st.t[0]]);
                    u.axis = saxis[pq.i];
                    u.lslot = pq.lslot;
                    u.gslot = sslot[pq.i];
                    u.c = std::cos(stheta[pq.i] / 2);
                    u.s = std::sin(stheta[pq.i] / 2);
                } else if (pq.kind == qsv::dev::SUB_U1) {
                    u.j = jpos(li[st.t[0]]);
                    u.mat = (int64_t)(mats.size() / 2);
                    for (const cd &v : qsv::dense_matrix(st)) push_c(v);
                } else if (pq.kind == qsv::dev::SUB_DIAG) {
                    u.mat = (int64_t)(mats.size() / 2);
                    for (int r = 0; r < 8; ++r) {
                        cd d(1, 0);
                        if ((r & u.cmask) == u.cmask) {
                            int idx = 0;
                            for (int q = 0; q < st.k; ++q)
                                idx |= ((r >> jpos(li[st.t[q]])) & 1) << q;
                            d = st.U[idx];
                        }
                        if (d != cd(1, 0)) u.touch |= 1u << r;
                        push_c(d);
                    }
                    u.cmask = 0;
                } else {   // SUB_PHASE
                    u.k = st.k;
                    u.touch = st.touch;
                    for (int q = 0; q < st.k; ++q) u.gt[q] = (uint32_t)st.t[q];
                    u.mat = (int64_t)(mats.size() / 2);
                    for (int r = 0; r < (1 << st.k); ++r) push_c(st.U[r]);
                }
                subs.push_back(u);
            }
            aops.push_back(a);
            ++L.count;
            bopen = false;
            bbits = 0;
            bq.clear();
            prev = -1;
        };
        for (int i : groups[gi].idx) {
            const bool rot = sslot[i] >= 0;
            if (rot && L.nrot == qsv::dev::kAdjMaxRot) {
                close_block();
                launches.push_back(L);
                L = Launch{gi, aops.size(), 0, 0};
                prev = -1;
            }
            const Op &st = steps[i];
            uint32_t lctrl = 0;
            uint64_t ectrl = 0;
            for (int p = 0; p < 64; ++p)
                if ((st.ctrl >> p) & 1) {
                    if (li[p] >= 0) lctrl |= 1u << li[p];
                    else ectrl |= 1ull << p;
                }
            const bool diag = st.kind == Op::MONO && st.diag;
            int nin = 0;
            uint32_t tin = 0;
            for (int j = 0; j < st.k; ++j)
                if (li[st.t[j]] >= 0) {
                    ++nin;
                    tin |= 1u << li[st.t[j]];
                }
            const bool outside = !rot && diag && nin == 0;
            if (use_blocks) {
                int kind = -1;
                if (rot) kind = qsv::dev::SUB_ROT;
                else if (outside) kind = qsv::dev::SUB_PHASE;
                else if (diag && nin == st.k) kind = qsv::dev::SUB_DIAG;
                else if (st.k == 1) kind = qsv::dev::SUB_U1;
                const uint32_t need = lctrl | (outside ? 0u : tin);
                if (kind == qsv::dev::SUB_PHASE && lctrl == 0 && !bopen) kind = -1;
                if (kind >= 0 && popc(need) <= 3) {
                    if (bopen && popc(bbits | need) > 3) close_block();
                    bopen = true;
                    bbits |= need;
                    bq.push_back(Pending{i, lctrl, ectrl, kind, rot ? L.nrot++ : -1});
                    continue;
                }
                close_block();
            }
            AdjOp a{};
            if (outside) {
                // diagonal, all targets outside the tile: a phase per tile
                qsv::dev::TileOp &t = a.op;
                t.k = st.k;
                t.touch = st.touch;
                for (int j = 0; j < st.k; ++j) t.gt[j] = (uint32_t)st.t[j];
                t.ectrl = ectrl;
                for (int b = 0; b < mt; ++b)
                    if (!((lctrl >> b) & 1)) t.fz[t.nfree++] = qsv::swz_elem(1u << b, eb) * eb;
                t.sl[0] = qsv::swz_elem(lctrl, eb) * eb;
                t.mat = (int64_t)(mats.size() / 2);
                for (int r = 0; r < (1 << st.k); ++r) push_c(st.U[r]);
                a.kind = qsv::dev::ADJ_PHASE;
                aops.push_back(a);
                ++L.count;
                prev = -1;
                continue;
            }
            if (rot && prev >= 0 && aops.back().nsub < qsv::dev::kAdjChain &&
                steps[prev].t[0] == st.t[0] && steps[prev].ctrl == st.ctrl) {
                AdjOp &ch = aops.back();
                const int j = ch.nsub++;
                ch.axis[j] = saxis[i];
                ch.lslot[j] = L.nrot++;
                ch.gslot[j] = sslot[i];
                ch.c[j] = std::cos(stheta[i] / 2);
                ch.s[j] = std::sin(stheta[i] / 2);
                continue;
            }
            a.op = qsv::lower_to_lds(st, li, mats, eb);
            if (rot) {
                a.kind = qsv::dev::ADJ_ROT;
                a.nsub = 1;
                a.axis[0] = saxis[i];
                a.lslot[0] = L.nrot++;
                a.gslot[0] = sslot[i];
                a.c[0] = std::cos(stheta[i] / 2);
                a.s[0] = std::sin(stheta[i] / 2);
                prev = i;
            } else {
                a.kind = qsv::dev::ADJ_APPLY;
                prev = -1;
            }
            aops.push_back(a);
            ++L.count;
        }
        close_block();
        if (L.count) launches.push_back(L);
    }
    if (launches.empty()) return QSV_OK;
    const size_t a_bytes = (aops.size() * sizeof(AdjOp) + 255) & ~size_t(255);
    const size_t u_bytes = (subs.size() * sizeof(qsv::dev::AdjSub) + 255) & ~size_t(255);
    const size_t nmat = mats.size();
    const size_t mat_bytes = s->opt.dtype == QSV_C128 ? nmat * sizeof(double) : nmat * sizeof(float);
    std::vector<unsigned char> host(a_bytes + u_bytes + mat_bytes + 16, 0);
    std::memcpy(host.data(), aops.data(), aops.size() * sizeof(AdjOp));
    if (!subs.empty())
        std::memcpy(host.data() + a_bytes, subs.data(), subs.size() * sizeof(qsv::dev::AdjSub));
    if (s->opt.dtype == QSV_C128) {
        if (nmat) std::memcpy(host.data() + a_bytes + u_bytes, mats.data(), mat_bytes);
    } else {
        float *f = reinterpret_cast<float *>(host.data() + a_bytes + u_bytes);
        for (size_t i = 0; i < nmat; ++i) f[i] = (float)mats[i];
    }
    void *dpool = nullptr;
    QSV_TRY(stage(s, host.data(), host.size(), &dpool));
    const AdjOp *daops = reinterpret_cast<const AdjOp *>(dpool);
    const qsv::dev::AdjSub *dsubs =
        reinterpret_cast<const qsv::dev::AdjSub *>((const unsigned char *)dpool + a_bytes);
    const void *dmat = (const unsigned char *)dpool + a_bytes + u_bytes;
    for (const Launch &L : launches) {
        const uint64_t tile = groups[L.group].tile;
        qsv::dev::TileArgs ta{};
        ta.m = popc(tile);
        ta.nq = n;
        ta.tile_pos_n = ta.m;
        ta.n_ops = (int)L.count;
        int c = 0;
        for (int p = 0; p < 64; ++p)
            if ((tile >> p) & 1) ta.tpos[c++] = (uint32_t)p;
        ta.n_tiles = 1ull << (n - ta.m);
        ta.mfma_k = mfma_k;
        for (int i = 0; i < 64 && (i << 8) < (1 << ta.m); ++i) {
            uint64_t d = 0;
            for (int b = 8; b < ta.m; ++b)
                if (((i << 8) >> b) & 1) d |= 1ull << ta.tpos[b];
            ta.dep_hi[i] = d;
        }
        const int tok = tbegin(s);
        QSV_HIP(s, qsv::dev::adjoint_tile_pass(s->opt.dtype, psi, phi, ta, daops + L.first, dsubs,
                                               dmat, L.nrot, partial, grid, s->stream));
        tend(s, tok, QSV_K_TILE, 4.0 * (double)s->dim() * s->elem());
        if (log_level() >= 2) {
            int nk[4] = {0, 0, 0, 0}, nsub = 0;
            for (size_t q = L.first; q < L.first + L.count; ++q) {
                ++nk[aops[q].kind];
                if (aops[q].kind == qsv::dev::ADJ_BLOCK) nsub += aops[q].nsub;
            }
            std::fprintf(stderr,
                         "qsv: adjoint pass tile=%#llx m=%d steps=%zu (apply %d, chains %d, "
                         "phases %d, blocks %d with %d sub-steps) rotations=%d\n",
                         (unsigned long long)tile, ta.m, L.count, nk[0], nk[1], nk[2], nk[3], nsub,
                         L.nrot);
        }
    }
    return QSV_OK;
}

}  // namespace

extern "C" qsv_status qsv_adjoint_gradient(qsv_sim *s, const qsv_circuit *circ,
                                           const qsv_pauli_sum *ham, double *value_out,
                                           double *grad_out) {
    QSV_CHECK(s);
    if (!circ || !ham || !value_out) return fail(s, QSV_EINVAL, "NULL argument");
    if (circ->n_qubits < 1 || circ->n_qubits > qsv::kMaxQubits || circ->n_gates < 0 ||
        (circ->n_gates > 0 && (!circ->op || !circ->k || !circ->c || !circ->qubits)) ||
        circ->n_params < 0 || (circ->n_params > 0 && !grad_out))
        return fail(s, QSV_EINVAL, "bad circuit description");
    if (ham->n_terms < 0 || (ham->n_terms > 0 && (!ham->xmask || !ham->zmask || !ham->coeff)))
        return fail(s, QSV_EINVAL, "bad Pauli sum");
    const int n = circ->n_qubits;
    const uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    for (int t = 0; t < ham->n_terms; ++t)
        if (((ham->xmask[t] | ham->zmask[t]) & ~full) != 0 || !std::isfinite(ham->coeff[t]))
            return fail(s, QSV_EINVAL, "Pauli term outside the circuit's qubits");
    const int G = circ->n_gates;
    std::vector<Gate> gates(G);
    std::vector<int> axis(G), param(G);
    int nrot = 0;
    for (int g = 0; g < G; ++g) {
        QSV_TRY(circuit_gate(s, circ, g, gates[g], &axis[g], &param[g]));
        if (axis[g]) ++nrot;
    }
    const uint64_t dim = 1ull << n;
    QSV_TRY(ensure_vectors(s, dim));
    if (!s->d_small) QSV_HIP(s, hipMalloc((void **)&s->d_small, 64 * sizeof(double)));
    void *psi = s->d_vec[0], *phi = s->d_vec[1];
    // partial sums per rotation: nb per workgroup-wave of the tiled sweep
    // (mode TILED), else per workgroup of the per-gate reverse kernels
    const bool tiled = s->opt.mode == QSV_MODE_TILED;
    int grid = 0, nb = 0, mfma_k = 0;
    if (tiled) {
        // widest step that may run on the matrix cores (dense, 3+ targets)
        for (int g = 0; g < G; ++g)
            if (!axis[g] && gates[g].k >= 3) mfma_k = std::max(mfma_k, gates[g].k);
        const int m = adjoint_tile_bits(s, n);
        grid = qsv::dev::adjoint_tile_grid(s->opt.dtype, m, mfma_k);
        if (grid < 1) return fail(s, QSV_EDEVICE, "adjoint tiles do not fit in LDS");
        grid = (int)std::min<uint64_t>((uint64_t)grid, 1ull << (n - m));
        nb = grid * qsv::dev::kAdjWaves;
    } else {
        nb = qsv::dev::adjoint_blocks(dim >> 1);
    }
    // workspace: [x z c ny | param order | grad | partials]
    const int T = ham->n_terms;
    const size_t off_z = 8 * (size_t)(T + 1), off_c = 16 * (size_t)(T + 1), off_ny = 24 * (size_t)(T + 1);
    const size_t off_po = (off_ny + 4 * (size_t)(T + 1) + 255) & ~size_t(255);
    const size_t off_gr = (off_po + 4 * (size_t)(nrot + 1) + 255) & ~size_t(255);
    const size_t off_pa = (off_gr + 8 * (size_t)(circ->n_params + 1) + 255) & ~size_t(255);
    // (the inner product <psi|H psi> uses up to 1024 partials after the rows)
    const size_t need = off_pa + 8 * ((size_t)nb * nrot + 1024) + 4096;
    QSV_TRY(ensure_ws(s, need));
    unsigned char *w = (unsigned char *)s->d_ws;
    std::vector<unsigned char> meta(off_gr, 0);
    std::vector<int32_t> ny(T + 1, 0), porder;
    // terms ordered by X mask (stable), so that the kernel gathers once per
    // distinct mask
    std::vector<int> tord(T);
    for (int t = 0; t < T; ++t) tord[t] = t;
    std::stable_sort(tord.begin(), tord.end(),
                     [&](int a, int b) { return ham->xmask[a] < ham->xmask[b]; });
    for (int q = 0; q < T; ++q) {
        const int t = tord[q];
        ny[q] = popc(ham->xmask[t] & ham->zmask[t]);
        std::memcpy(meta.data() + 8 * (size_t)q, &ham->xmask[t], 8);
        std::memcpy(meta.data() + off_z + 8 * (size_t)q, &ham->zmask[t], 8);
        std::memcpy(meta.data() + off_c + 8 * (size_t)q, &ham->coeff[t], 8);
    }
    if (T) std::memcpy(meta.data() + off_ny, ny.data(), 4 * T);
    for (int g = G - 1; g >= 0; --g)
        if (axis[g]) porder.push_back(param[g]);
    if (!porder.empty()) std::memcpy(meta.data() + off_po, porder.data(), 4 * porder.size());
    QSV_HIP(s, hipMemcpyAsync(w, meta.data(), off_gr, hipMemcpyHostToDevice, s->stream));

    StateSwap sw(s, psi, n);
    // forward: psi = U|0>
    QSV_HIP(s, qsv::dev::fill_basis0(s->opt.dtype, psi, dim, s->stream));
    {
        std::vector<Op> ops;
        for (const Gate &g : gates) {
            Op op;
            if (qsv::canonicalize(g, op)) ops.push_back(std::move(op));
        }
        QSV_TRY(run_ops(s, ops));
    }
    // phi = H psi, value = Re<psi|phi>
    QSV_HIP(s, qsv::dev::ham_apply(s->opt.dtype, psi, phi, dim, T, (const uint64_t *)w,
                                   (const uint64_t *)(w + off_z), (const double *)(w + off_c),
                                   (const int32_t *)(w + off_ny), s->stream));
    double *partial = (double *)(w + off_pa);
    QSV_HIP(s, qsv::dev::dot_re(s->opt.dtype, psi, phi, dim, partial + (size_t)nb * nrot,
                                s->d_small, s->stream));
    // reverse sweep
    if (tiled)
        QSV_TRY(adjoint_reverse_tiled(s, gates, axis, circ->params, param, psi, phi, partial, grid,
                                      mfma_k));
    int slot = 0;
    for (int g = G - 1; g >= 0 && !tiled; --g) {
        const Gate &gt = gates[g];
        if (axis[g]) {
            const int c = popc(gt.ctrl);
            qsv::dev::IndexArgs ia;
            index_args((1ull << gt.t[0]) | gt.ctrl, gt.ctrl, ia);
            const double th = circ->params[param[g]];
            const int tok = tbegin(s);
            QSV_HIP(s, qsv::dev::adjoint_rotation(s->opt.dtype, psi, phi, dim >> (1 + c), ia,
                                                  1ull << gt.t[0], axis[g], std::cos(th / 2),
                                                  std::sin(th / 2), partial + (size_t)nb * slot,
                                                  nb, s->stream));
            tend(s, tok, QSV_K_DENSE, 4.0 * (double)(dim >> c) * s->elem());
            ++slot;
        } else {
            Gate d = gt;
            const int D = 1 << gt.k;
            for (int r = 0; r < D; ++r)
                for (int cc = 0; cc < D; ++cc) d.U[(size_t)r * D + cc] = std::conj(gt.U[(size_t)cc * D + r]);
            Op op;
            if (!qsv::canonicalize(d, op)) continue;
            sw.to(psi);
            QSV_TRY(launch_op(s, op));
            sw.to(phi);
            QSV_TRY(launch_op(s, op));
        }
    }
    double *dgrad = (double *)(w + off_gr);
    if (circ->n_params > 0) {
        QSV_HIP(s, qsv::dev::grad_finish(partial, nrot, nb, (const int32_t *)(w + off_po), dgrad,
                                         circ->n_params, s->stream));
        QSV_HIP(s, hipMemcpyAsync(grad_out, dgrad, 8 * (size_t)circ->n_params,
                                  hipMemcpyDeviceToHost, s->stream));
    }
    QSV_HIP(s, hipMemcpyAsync(value_out, s->d_small, sizeof(double), hipMemcpyDeviceToHost,
                              s->stream));
    return sync(s);
}
