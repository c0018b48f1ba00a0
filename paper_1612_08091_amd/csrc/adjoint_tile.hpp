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
enum AdjKind { ADJ_APPLY = 0, ADJ_ROT = 1, ADJ_PHASE = 2 };
struct AdjOp {
    TileOp op;
    int32_t kind;
    int32_t nsub;
    int32_t axis[kAdjChain];
    int32_t lslot[kAdjChain];
    int32_t gslot[kAdjChain];
    int32_t pad;
    double c[kAdjChain];
    double s[kAdjChain];
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
// (widest matrix-core step of the sweep) as for the forward LDS tile kernel; `ops` are ta.n_ops steps in order, holding at most
// kAdjMaxRot rotations (lslot 0..nrot-1, each used once); `pool` the
// matrices in the state's complex type.  Writes
// partial[gslot * nb + 4 * block + wave] for every rotation of the pass,
// nb = 4 * grid.
hipError_t adjoint_tile_pass(int dtype, void *psi, void *phi, const TileArgs &ta,
                             const AdjOp *ops, const void *pool, int nrot, double *partial,
                             int grid, hipStream_t s);

}  // namespace dev
}  // namespace qsv
