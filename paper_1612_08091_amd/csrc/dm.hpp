// Reductions over a density matrix held as vec(rho) on 2n qubits
// (rho[r][c] at index r + 2^n c).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsv {
namespace dev {

// out[i] = Re v[i + (i << n)] for i < 2^n (device memory).
hipError_t dm_diagonal(int dtype, const void *v, int n, double *out, hipStream_t s);

// For each term t: part[2 t], part[2 t + 1] = sum_r (-1)^popcount(r & z_t)
// v[r + ((r ^ x_t) << n)] (real, imaginary), r < 2^n; one workgroup per
// term.  x, z: device arrays of nterms masks; part: 2 nterms doubles.
hipError_t dm_pauli_sums(int dtype, const void *v, int n, int nterms, const uint64_t *x,
                         const uint64_t *z, double *part, hipStream_t s);

}  // namespace dev
}  // namespace qsv
