// Tiled reverse sweep of the adjoint gradient (Jones and Gacon, 2020).
//
// The reverse sweep applies U_g^dagger to two vectors, psi and phi, for every
// gate g from the last to the first, and at each rotation gate
// exp(-i theta P / 2) first records Im<phi|P|psi>.  Every step acts on a few
// qubits, so the same planning as the forward tile passes applies: a pass
// loads the psi and phi tiles of 2^m amplitudes that share the bits outside
// the tile, runs all of the pass's steps in LDS and writes both tiles back.
// The inner products split over tiles: each workgroup accumulates its tiles'
// share per wave and rotation and writes it out once per pass; the host sums
// these partials in a fixed order, so the gradient is the same from run to
// run (tiles are assigned to workgroups statically).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace qsv {
namespace dev {

constexpr int kAdjChain = 4;            // rotations fused into one step

// One reverse step on both tiles.
//  kind ADJ_APPLY: apply `op` (U^dagger of a gate, lowered like a forward
//    tile op) to the psi tile and to the phi tile.
//  kind ADJ_ROT: a chain of nsub rotations exp(-i theta_j P_j / 2) on one
//    target with the same controls, in reverse order: for j = 0..nsub-1,
//    record Im<phi|P_j|psi> on the pairs `op` addresses (a dense one-target
//    op: fz, sl, nfree, ectrl), then apply
//    U_j^dagger = cos(theta_j/2) + i sin(theta_j/2) P_j to both tiles.
//    axis 1, 2, 3 = X, Y, Z; lslot is the rotation's accumulator within the
//    launch, gslot its row in the partial array.
//  kind ADJ_PHASE: a diagonal op (MONO, k targets) whose targets all lie
//    outside the tile: op.gt holds the targets' global positions, op.touch
//    the rows that change, op.ectrl the controls outside the tile, and
//    op.fz / op.sl[0] / op.nfree address the amplitudes whose in-tile
//    control bits are set (nfree = m: no in-tile controls); the pool holds
//    the 2^k diagonal values at op.mat.
//  kind ADJ_BLOCK: nsub sub-steps (AdjSub sub0 .. sub0 + nsub - 1) on three
//    tile bits, the block: each thread loads the 8 amplitudes of a group
//    (op.sl[0..7] the block rows, op.fz / op.nfree the other tile bits) of
//    both tiles, runs the sub-steps on them in registers and stores them.
enum AdjKind { ADJ_APPLY = 0, ADJ_ROT = 1, ADJ_PHASE = 2, ADJ_BLOCK = 3 };
struct AdjOp {
    TileOp op;
    int32_t kind;
    int32_t nsub;
    int32_t axis[kAdjChain];
    int32_t lslot[kAdjChain];
    int32_t gslot[kAdjChain];
    int32_t sub0;
    double c[kAdjChain];
    double s[kAdjChain];
};

// Sub-steps of a block, on block rows r = 0..7 (bit j of r = block bit j):
//  SUB_ROT: rotation about `axis` on block bit j (as in a chain), on the
//    pairs whose rows contain cmask; lslot / gslot as for chains.
//  SUB_U1: the 2x2 matrix at pool[mat] on block bit j, rows containing cmask.
//  SUB_DIAG: row r multiplied by pool[mat + r] for the rows in `touch`.
//  SUB_PHASE: a diagonal op with k targets outside the tile: row index
//    r_out from the tile base's bits gt[0..k-1]; if r_out is in `touch`, the
//    rows containing cmask are multiplied by pool[mat + r_out] (cmask = 0:
//    the whole tile, recorded as a pending phase).
//  All: skipped on tiles whose base lacks one of the ectrl bits.
enum AdjSubKind { SUB_ROT = 0, SUB_U1 = 1, SUB_DIAG = 2, SUB_PHASE = 3 };
struct AdjSub {
    int32_t kind;
    int32_t j;
    int32_t cmask;
    int32_t axis;
    int32_t lslot;
    int32_t gslot;
    int32_t k;
    uint32_t touch;
    uint32_t gt[6];
    uint64_t ectrl;
    double c, s;
    int64_t mat;
};

constexpr int kAdjWaves = 4;            // waves per workgroup (256 threads)
constexpr int kAdjMaxRot = 256;         // rotations per launch (LDS accumulators)

// Dynamic LDS bytes of one workgroup: the two tiles and the accumulators.
inline size_t adjoint_tile_lds(int dtype, int m) {
    return 2 * ((dtype == 0 ? 16u : 8u) << m) + 8u * kAdjWaves * kAdjMaxRot;
}

// Workgroups that fit on the device at once for tile bits m and the widest
// matrix-core step mfma_k (0: none) of the sweep (the grid of every launch
// of one sweep); 0 if the tiles do not fit in LDS.
int adjoint_tile_grid(int dtype, int m, int mfma_k);

// One pass: ta.m, ta.n_ops, ta.tpos, ta.n_tiles, ta.dep_hi and ta.mfma_k
// (widest matrix-core step of the sweep) as for the forward LDS tile
// kernel; `ops` are ta.n_ops steps in order, holding at most kAdjMaxRot
// rotations (lslot 0..nrot-1, each used once); `subs` the sub-steps of
// their blocks; `pool` the matrices in the state's complex type.  Writes
// partial[gslot * nb + 4 * block + wave] for every rotation of the pass,
// nb = 4 * grid.
hipError_t adjoint_tile_pass(int dtype, void *psi, void *phi, const TileArgs &ta,
                             const AdjOp *ops, const AdjSub *subs, const void *pool, int nrot,
                             double *partial, int grid, hipStream_t s);

}  // namespace dev
}  // namespace qsv
