// Emulated math gates (ProjectQ Sec. 4.3.3): a tabulated classical bijection
// applied to the value of a qubit register across the whole state.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsv {
namespace dev {

constexpr int kMaxMathBits = 26;

// Register and controls as global bit positions.  shift >= 0: the register
// is the contiguous bits shift .. shift + w - 1 (pos ignored).
struct MathArgs {
    uint64_t regmask;
    uint64_t ctrl;
    int32_t w;
    int32_t shift;
    uint32_t pos[kMaxMathBits];
};

// out[j] = in[src(j)]: for j with all control bits set, src(j) is j with the
// register value y replaced by inv[y] (inv = the table's inverse, 2^w
// entries, device memory); src(j) = j otherwise.  in and out must not
// overlap.  dim = 2^n amplitudes of the state's complex type.
hipError_t math_gather(int dtype, const void *in, void *out, uint64_t dim, const MathArgs &a,
                       const uint32_t *inv, hipStream_t s);

}  // namespace dev
}  // namespace qsv
