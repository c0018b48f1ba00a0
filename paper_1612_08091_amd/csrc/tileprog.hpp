// Lowering of planned passes to tile-kernel instruction lists.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "device.hpp"
#include "qsv_internal.hpp"

namespace qsv {

struct TileProgram {
    uint64_t tile = 0;
    int m = 0;
    bool reg = false;                   // register-resident kernel (else LDS kernel)
    std::vector<dev::RegOp> rops;       // register kernel instructions
    std::vector<dev::TileOp> lops;      // LDS ops (all ops of an LDS-kernel pass)
    uint8_t reg_lbit[8] = {};           // initial layout (register kernel)
    uint8_t thr_lbit[16] = {};
    uint64_t g_reg[8] = {};             // initial layout as global index bits
    uint64_t g_thr[16] = {};
    uint64_t g_reg_f[8] = {};           // layout at store time
    uint64_t g_thr_f[16] = {};
    std::vector<unsigned char> img;     // LDS image (register kernel): tables, lane words
    bool permutes = false;              // stores to relabeled positions (Pass::dest)
    bool store_sync = false;            // workgroup barrier between the ops and the stores
                                        // (threads store amplitudes other threads loaded)
    uint8_t spos[64] = {};              // store position of each tile bit
    int remaps = 0;                     // layout changes through LDS
    int local_remaps = 0;               // of which within each wave (no workgroup barrier)
    int diag_merged = 0;                // diagonal ops folded into another
    int real_ops = 0;                   // register ops split into phases x real matrix
    int diag_ops = 0;                   // DIAG ops of the register program
    int mfma_k = 0;                     // widest matrix-core op (LDS kernel)
    double flops_per_amp = 0.0;
};

// Lower pass `ps` for a register kernel with rb register bits (rb = 0: LDS
// kernel).  The register kernel is used when the tile has rb + 8 bits
// (256 threads) or rb + 9 bits (512 threads, rb <= 4).
// Matrices are appended to `mats` as complex128 (re, im) pairs; ops refer to
// them by complex-entry offset.  elem_bytes (16 or 8, the state's complex
// type) fixes the LDS byte offsets of the remaps.
void compile_pass(const Pass &ps, int rb, std::vector<double> &mats, TileProgram &prog,
                  int elem_bytes = 16);

// Swizzled element index of local index l in an LDS tile (the same XOR
// swizzle as the device's swz<R>: the bits above the 256-byte bank span are
// folded into the bits below it); elem_bytes is 16 or 8.
uint32_t swz_elem(uint32_t l, int elem_bytes);

// Byte offset in the half-tile remap buffer of local index l when local bit
// `kept` (the one that stays in its register slot) is dropped: the compacted
// index, XOR-swizzled against bank conflicts, times elem_bytes.  Linear over
// GF(2) in l.
uint32_t remap_offset(uint32_t l, int kept, int elem_bytes);

// Real split of a k-qubit matrix (Sec. 4.3.2's fused gates, applied with less
// arithmetic): find unit-modulus l[r], rr[c] with U[r][c] = l[r] M[r][c] rr[c]
// and M real (up to an imaginary residue of 1e-14 per entry, dropped).
// Returns false when no such split exists.
bool real_split(const std::vector<cd> &U, int k, std::vector<cd> &l, std::vector<double> &M,
                std::vector<cd> &rr);

// Host model of the register-resident tile kernel: runs the program of a
// lowered pass on every tile of `state` (2^n complex amplitudes, in place),
// thread by thread and register by register, with the kernel's layouts, LDS
// byte offsets and image lookups, each bounds-checked.  A check of the
// lowering on the CPU; no product path calls it.  Returns "" on success, else
// the first violation found.
std::string emulate_reg_pass(const TileProgram &prog, int rb, const std::vector<double> &mats,
                             int elem_bytes, int n, std::vector<cd> &state);

// LDS-kernel form of one op; li maps a global bit position to its tile bit
// (-1 outside the tile); elem_bytes is the state's complex size (16 or 8).
dev::TileOp lower_to_lds(const Op &op, const int *li, std::vector<double> &mats, int elem_bytes);

}  // namespace qsv
