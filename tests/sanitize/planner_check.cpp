// Drives the host side of the tile path -- gate canonicalisation, fusion,
// pass planning with and without relabeling, lowering to register-kernel
// programs and LDS-kernel ops, and the host model of the register kernel --
// on small seeded circuits, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer.  The states from the host model are checked
// against a direct gate-by-gate application.  Prints "ok" and returns 0.
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "qsv_internal.hpp"
#include "tileprog.hpp"

using namespace qsv;

static void apply_direct(std::vector<cd> &psi, const Op &op) {
    const std::vector<cd> U = dense_matrix(op);
    const int D = 1 << op.k;
    std::vector<cd> in(D);
    for (uint64_t i = 0; i < psi.size(); ++i) {
        bool base = (i & op.ctrl) == op.ctrl;
        for (int j = 0; j < op.k && base; ++j)
            if ((i >> op.t[j]) & 1) base = false;
        if (!base) continue;
        for (int c = 0; c < D; ++c) {
            uint64_t x = i;
            for (int j = 0; j < op.k; ++j)
                if ((c >> j) & 1) x |= 1ull << op.t[j];
            in[c] = psi[x];
        }
        for (int r = 0; r < D; ++r) {
            cd acc = 0;
            for (int c = 0; c < D; ++c) acc += U[(size_t)r * D + c] * in[c];
            uint64_t x = i;
            for (int j = 0; j < op.k; ++j)
                if ((r >> j) & 1) x |= 1ull << op.t[j];
            psi[x] = acc;
        }
    }
}

static std::vector<cd> rand_unitary(int d, std::mt19937_64 &g) {
    std::normal_distribution<double> N;
    std::vector<cd> u((size_t)d * d);
    for (auto &x : u) x = cd(N(g), N(g));
    for (int c = 0; c < d; ++c) {
        for (int p = 0; p < c; ++p) {
            cd dot = 0;
            for (int r = 0; r < d; ++r) dot += std::conj(u[(size_t)r * d + p]) * u[(size_t)r * d + c];
            for (int r = 0; r < d; ++r) u[(size_t)r * d + c] -= dot * u[(size_t)r * d + p];
        }
        double nn = 0;
        for (int r = 0; r < d; ++r) nn += std::norm(u[(size_t)r * d + c]);
        nn = std::sqrt(nn);
        for (int r = 0; r < d; ++r) u[(size_t)r * d + c] /= nn;
    }
    return u;
}

int main() {
    std::mt19937_64 g(11);
    int bad = 0, programs = 0, lds = 0;
    for (int trial = 0; trial < 12; ++trial) {
        const int n = 12 + trial % 3;
        std::vector<Op> ops;
        std::uniform_int_distribution<int> pick(0, n - 1);
        for (int i = 0; i < 80; ++i) {
            Gate ga;
            const int kind = i % 6;
            ga.k = (kind == 3 && trial % 4 == 0) ? 3 : (kind == 1 || kind == 3 || kind == 4 ? 2 : 1);
            std::vector<int> qs;
            while ((int)qs.size() < ga.k + 1) {
                const int q = pick(g);
                bool dup = false;
                for (int x : qs) dup = dup || x == q;
                if (!dup) qs.push_back(q);
            }
            for (int j = 0; j < ga.k; ++j) ga.t[j] = qs[j];
            if (kind == 2 || kind == 5) ga.ctrl = 1ull << qs[ga.k];
            if (kind == 5) {   // a diagonal phase
                ga.U = {1, 0, 0, std::polar(1.0, 0.3 * i)};
            } else if (kind == 4) {   // a swap
                ga.U = {1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, 1};
            } else {
                ga.U = rand_unitary(1 << ga.k, g);
            }
            Op o;
            if (canonicalize(ga, o)) ops.push_back(o);
        }
        std::vector<cd> psi0(1ull << n);
        std::normal_distribution<double> N;
        for (auto &x : psi0) x = cd(N(g), N(g));
        std::vector<cd> want = psi0;
        for (const Op &o : ops) apply_direct(want, o);
        for (int k_max : {1, 2, 3}) {
            for (bool relabel : {false, true}) {
                const int m = 12, rb = 4;
                std::vector<Pass> passes = plan_tiled(ops, n, m, k_max, 9, relabel);
                // relabeling: each pass permutes positions inside its tile
                // only, and the passes together leave every qubit home
                int at[64];
                for (int p = 0; p < 64; ++p) at[p] = p;
                for (const Pass &ps : passes) {
                    if (ps.dest.empty()) continue;
                    if ((int)ps.dest.size() != n) {
                        std::fprintf(stderr, "dest of size %zu for %d qubits\n", ps.dest.size(), n);
                        return 1;
                    }
                    uint64_t img = 0;
                    for (int p = 0; p < n; ++p) {
                        const int d = ps.dest[p];
                        const bool in = (ps.tile >> p) & 1;
                        if ((!in && d != p) || (in && !((ps.tile >> d) & 1)) || ((img >> d) & 1)) {
                            std::fprintf(stderr, "dest is not a permutation of the tile\n");
                            return 1;
                        }
                        img |= 1ull << d;
                    }
                    int nat[64];
                    for (int p = 0; p < 64; ++p) nat[p] = at[p];
                    for (int p = 0; p < n; ++p) nat[ps.dest[p]] = at[p];
                    for (int p = 0; p < 64; ++p) at[p] = nat[p];
                }
                for (int p = 0; p < n; ++p)
                    if (at[p] != p) {
                        std::fprintf(stderr, "qubit %d ends at position %d\n", at[p], p);
                        return 1;
                    }
                std::vector<cd> psi = psi0;
                bool all_reg = true;
                for (const Pass &ps : passes) {
                    std::vector<double> mats;
                    TileProgram pg;
                    compile_pass(ps, rb, mats, pg, 16);
                    ++programs;
                    if (!pg.reg) {
                        all_reg = false;
                        ++lds;
                        continue;
                    }
                    const std::string err = emulate_reg_pass(pg, rb, mats, 16, n, psi);
                    if (!err.empty()) {
                        std::fprintf(stderr, "host model: %s\n", err.c_str());
                        return 1;
                    }
                }
                // the plan's ops on their own positions reproduce the state
                std::vector<cd> flat = psi0;
                for (const Op &o : pass_ops_in_qubit_order(passes, n)) apply_direct(flat, o);
                double d = 0, e = 0;
                for (size_t i = 0; i < want.size(); ++i) {
                    d = std::max(d, std::abs(flat[i] - want[i]));
                    if (all_reg) e = std::max(e, std::abs(psi[i] - want[i]));
                }
                if (d > 1e-10 || e > 1e-10) {
                    std::fprintf(stderr, "trial %d k_max %d relabel %d: plan %.3g model %.3g\n",
                                 trial, k_max, (int)relabel, d, e);
                    ++bad;
                }
            }
        }
    }
    if (bad) return 1;
    std::printf("ok (%d programs, %d on the LDS kernel)\n", programs, lds);
    return 0;
}
