/*
 * qsv_oracle.c -- plain, slow, obviously correct CPU reference of the
 * state-vector simulator's hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * path.
 *
 * What it computes (ProjectQ, Sec. 4.3.2: the simulator applies individual
 * gates to the full state; Sec. 4.1.3: a Control block conditions on the
 * control qubits being |1>; Sec. 4 and App. A: measurement in the
 * computational basis; Sec. 4.1.1: deallocating a qubit in superposition is
 * an error):
 *
 *   state      psi[i], i = sum_q b_q 2^q, complex128 stored as (re, im) pairs;
 *              qubit q is bit q of the index.
 *   gate       (U, targets[k], controls[c]): for every index i whose target
 *              bits are 0 and whose control bits are all 1,
 *                  out[i + off(r)] = sum_col U[r][col] psi[i + off(col)],
 *              off(r) = sum_j bit_j(r) 2^{targets[j]}; every other amplitude
 *              is left as it is.
 *   reductions sequential left-to-right sums in double precision.
 *
 * Built with gcc -O2 -ffp-contract=off -fopenmp.  Single-threaded unless
 * oracle_set_threads asks for more: then only the outer loop of
 * oracle_apply (over the independent index groups of one gate, each written
 * by one thread) is shared out, which changes no result.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 1;

/* Threads for oracle_apply's outer loop (1 = serial, the default).
 * Returns the number in effect. */
int oracle_set_threads(int t)
{
#ifdef _OPENMP
    g_threads = t < 1 ? 1 : t;
#else
    (void)t;
    g_threads = 1;
#endif
    return g_threads;
}

static int bit_of(uint64_t i, int q) { return (int)((i >> q) & 1u); }

/* Apply one (controlled) k-qubit gate.  Returns 0, or -1 on bad arguments. */
int oracle_apply(double *psi_d, int n, const double *u_d, int k,
                 const int *targets, int nc, const int *controls)
{
    if (k < 1 || k > 10 || n < k + nc) return -1;
    cplx *psi = (cplx *)psi_d;
    const cplx *u = (const cplx *)u_d;
    const uint64_t dim = (uint64_t)1 << n;
    const int blk = 1 << k;
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * blk);
    if (!off) return -1;
    for (int r = 0; r < blk; ++r) {
        uint64_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((r >> j) & 1) o += (uint64_t)1 << targets[j];
        off[r] = o;
    }
    int failed = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(g_threads) reduction(| : failed)
#endif
    {
        cplx *in = (cplx *)malloc(sizeof(cplx) * blk);
        cplx *out = (cplx *)malloc(sizeof(cplx) * blk);
        if (!in || !out) failed = 1;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (uint64_t i = 0; i < dim; ++i) {
            int ok = !failed;
            for (int j = 0; ok && j < k; ++j)
                if (bit_of(i, targets[j])) ok = 0;
            for (int j = 0; ok && j < nc; ++j)
                if (!bit_of(i, controls[j])) ok = 0;
            if (!ok) continue;
            for (int c = 0; c < blk; ++c) in[c] = psi[i + off[c]];
            for (int r = 0; r < blk; ++r) {
                cplx acc = 0;
                for (int c = 0; c < blk; ++c) acc += u[(size_t)r * blk + c] * in[c];
                out[r] = acc;
            }
            for (int r = 0; r < blk; ++r) psi[i + off[r]] = out[r];
        }
        free(in);
        free(out);
    }
    free(off);
    return failed ? -1 : 0;
}

/* p_i = |psi_i|^2 */
void oracle_probs(const double *psi_d, int n, double *out)
{
    const cplx *psi = (const cplx *)psi_d;
    const uint64_t dim = (uint64_t)1 << n;
    for (uint64_t i = 0; i < dim; ++i) {
        double re = creal(psi[i]), im = cimag(psi[i]);
        out[i] = re * re + im * im;
    }
}

/* sum of p_i over the indices whose bit qubits[j] equals bits[j] for all j */
double oracle_prob_bits(const double *psi_d, int n, int m, const int *qubits,
                        const int *bits)
{
    const cplx *psi = (const cplx *)psi_d;
    const uint64_t dim = (uint64_t)1 << n;
    double s = 0.0;
    for (uint64_t i = 0; i < dim; ++i) {
        int ok = 1;
        for (int j = 0; j < m; ++j)
            if (bit_of(i, qubits[j]) != (bits[j] ? 1 : 0)) { ok = 0; break; }
        if (!ok) continue;
        double re = creal(psi[i]), im = cimag(psi[i]);
        s += re * re + im * im;
    }
    return s;
}

/* Entry (a, b) of the single-qubit Pauli matrix with letter code
 * 0 = I, 1 = X, 2 = Z, 3 = Y  (code = xbit + 2*zbit). */
static cplx pauli_entry(int code, int a, int b)
{
    switch (code) {
    case 0: return a == b ? 1.0 : 0.0;
    case 1: return a != b ? 1.0 : 0.0;
    case 2: return a == b ? (a ? -1.0 : 1.0) : 0.0;
    default: /* Y = [[0, -i], [i, 0]] */
        if (a == b) return 0.0;
        return a == 0 ? -I : I;
    }
}

/* <psi| P_t |psi> for every term t of a Pauli sum, P_t = tensor over qubits of
 * single-qubit Paulis (letter on qubit q from bit q of xmask/zmask).
 * (P psi)_j = sum_i P[j][i] psi_i with P[j][i] = prod_q sigma_q[j_q][i_q];
 * only i = j ^ xmask is nonzero.  Writes each term's complex value to
 * term_out (2 doubles per term) if non-NULL and returns sum_t coeff_t Re<P_t>;
 * *imag_out receives sum_t coeff_t Im<P_t>. */
double oracle_expectation(const double *psi_d, int n, int nterms,
                          const uint64_t *xmask, const uint64_t *zmask,
                          const double *coeff, double *term_out, double *imag_out)
{
    const cplx *psi = (const cplx *)psi_d;
    const uint64_t dim = (uint64_t)1 << n;
    double tot_re = 0.0, tot_im = 0.0;
    int *sup = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int *code = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int t = 0; t < nterms; ++t) {
        int w = 0;
        for (int q = 0; q < n; ++q) {
            int c = (int)((xmask[t] >> q) & 1u) + 2 * (int)((zmask[t] >> q) & 1u);
            if (c) { sup[w] = q; code[w] = c; ++w; }
        }
        cplx acc = 0;
        for (uint64_t j = 0; j < dim; ++j) {
            uint64_t i = j ^ xmask[t];
            cplx f = 1.0;
            for (int s = 0; s < w; ++s)
                f *= pauli_entry(code[s], bit_of(j, sup[s]), bit_of(i, sup[s]));
            acc += conj(psi[j]) * f * psi[i];
        }
        if (term_out) { term_out[2 * t] = creal(acc); term_out[2 * t + 1] = cimag(acc); }
        tot_re += coeff[t] * creal(acc);
        tot_im += coeff[t] * cimag(acc);
    }
    free(sup); free(code);
    if (imag_out) *imag_out = tot_im;
    return tot_re;
}

/* Measure qubit q with the caller's uniform u in [0,1):
 * p0 = sum over bit q = 0, p1 = sum over bit q = 1, T = p0 + p1;
 * outcome 0 iff u*T < p0.  The other branch is zeroed and the kept one is
 * scaled by 1/sqrt(p_outcome).  Returns the outcome; probs_out gets (p0, p1). */
int oracle_measure(double *psi_d, int n, int q, double u, double *probs_out)
{
    cplx *psi = (cplx *)psi_d;
    const uint64_t dim = (uint64_t)1 << n;
    double p0 = 0.0, p1 = 0.0;
    for (uint64_t i = 0; i < dim; ++i) {
        double re = creal(psi[i]), im = cimag(psi[i]);
        if (bit_of(i, q)) p1 += re * re + im * im;
        else p0 += re * re + im * im;
    }
    double total = p0 + p1;
    int outcome = (u * total < p0) ? 0 : 1;
    double keep = outcome ? p1 : p0;
    double scale = 1.0 / sqrt(keep);
    for (uint64_t i = 0; i < dim; ++i) {
        if (bit_of(i, q) == outcome) psi[i] *= scale;
        else psi[i] = 0;
    }
    if (probs_out) { probs_out[0] = p0; probs_out[1] = p1; }
    return outcome;
}

/* Sampling without collapse: C_i = sum_{j<=i} p_j (sequential), T = C_last;
 * shot s returns the smallest i with C_i > u_s * T, or, if there is none, the
 * largest i with p_i > 0. */
int oracle_sample(const double *psi_d, int n, int shots, const double *u, uint64_t *out)
{
    const cplx *psi = (const cplx *)psi_d;
    const uint64_t dim = (uint64_t)1 << n;
    double *cdf = (double *)malloc(sizeof(double) * dim);
    if (!cdf) return -1;
    double run = 0.0;
    uint64_t last_nz = 0;
    for (uint64_t i = 0; i < dim; ++i) {
        double re = creal(psi[i]), im = cimag(psi[i]);
        double p = re * re + im * im;
        if (p > 0.0) last_nz = i;
        run += p;
        cdf[i] = run;
    }
    for (int s = 0; s < shots; ++s) {
        double r = u[s] * run;
        uint64_t lo = 0, hi = dim; /* first index with cdf > r in [lo, hi) */
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > r) hi = mid; else lo = mid + 1;
        }
        out[s] = (lo < dim) ? lo : last_nz;
    }
    free(cdf);
    return 0;
}

/* Remove qubit q if it is classical: p1 <= tau -> value 0, p0 <= tau -> value 1,
 * otherwise return -1 and leave out untouched.  out (2^(n-1) amplitudes) gets
 * the kept half, compacted: out[i'] = psi[i' with bit `value` inserted at q]. */
int oracle_dealloc(const double *psi_d, int n, int q, double tau, double *out_d)
{
    const cplx *psi = (const cplx *)psi_d;
    cplx *out = (cplx *)out_d;
    const uint64_t dim = (uint64_t)1 << n;
    double p0 = 0.0, p1 = 0.0;
    for (uint64_t i = 0; i < dim; ++i) {
        double re = creal(psi[i]), im = cimag(psi[i]);
        if (bit_of(i, q)) p1 += re * re + im * im;
        else p0 += re * re + im * im;
    }
    int value;
    if (p1 <= tau) value = 0;
    else if (p0 <= tau) value = 1;
    else return -1;
    const uint64_t half = dim >> 1;
    const uint64_t low = ((uint64_t)1 << q) - 1;
    for (uint64_t j = 0; j < half; ++j) {
        uint64_t i = ((j & ~low) << 1) | (j & low) | ((uint64_t)value << q);
        out[j] = psi[i];
    }
    return value;
}

/* Emulated math gate (Sec. 4.3.3: a gate deriving from BasicMathGate applies
 * a classical function to a superposition of register values directly,
 * instead of its decomposition into 1- and 2-qubit gates).  The register is
 * qubits[0..w-1], qubits[0] the least significant bit; f is tabulated as
 * table[x] for x = 0..2^w-1 and must be a bijection (else -1: the map would
 * not be unitary).  For every index i whose control bits are all 1, the
 * amplitude psi[i] moves to the index that holds the register value
 * table[x(i)] and the same other bits; every other amplitude stays. */
int oracle_apply_math(double *psi_d, int n, int w, const int *qubits,
                      const uint32_t *table, int nc, const int *controls)
{
    if (w < 1 || w > 30 || n < w + nc) return -1;
    cplx *psi = (cplx *)psi_d;
    const uint64_t dim = (uint64_t)1 << n;
    const uint64_t size = (uint64_t)1 << w;
    unsigned char *seen = (unsigned char *)calloc(size, 1);
    cplx *out = (cplx *)malloc(sizeof(cplx) * dim);
    if (!seen || !out) { free(seen); free(out); return -1; }
    for (uint64_t x = 0; x < size; ++x) {
        if (table[x] >= size || seen[table[x]]) { free(seen); free(out); return -1; }
        seen[table[x]] = 1;
    }
    for (uint64_t i = 0; i < dim; ++i) {
        int ok = 1;
        for (int j = 0; j < nc; ++j)
            if (!bit_of(i, controls[j])) ok = 0;
        if (!ok) { out[i] = psi[i]; continue; }
        uint64_t x = 0, rest = i;
        for (int b = 0; b < w; ++b) {
            x |= (uint64_t)bit_of(i, qubits[b]) << b;
            rest &= ~((uint64_t)1 << qubits[b]);
        }
        const uint64_t y = table[x];
        uint64_t j = rest;
        for (int b = 0; b < w; ++b)
            if ((y >> b) & 1) j |= (uint64_t)1 << qubits[b];
        out[j] = psi[i];
    }
    memcpy(psi, out, sizeof(cplx) * dim);
    free(seen); free(out);
    return 0;
}

/* ------------------------------------------------------------------------
 * Density matrices (Sec. 4.3.2 names a density-matrix simulator for noise as
 * future work).  rho is 2^n x 2^n, row-major, rho[r * 2^n + c].
 * ---------------------------------------------------------------------- */

/* rho <- G rho G^dagger for the (controlled) gate G = (U, targets, controls)
 * on n qubits, or rho <- sum_j K_j rho K_j^dagger over nk Kraus matrices
 * (kraus_d: nk matrices of 2^k x 2^k, controls ignored when nk > 1).  Both
 * are written out from the definition: G (or K_j) is applied to every column
 * of rho, then to every column of the conjugate transpose of the result.
 * Returns 0, or -1 on bad arguments. */
static int dm_conjugate(cplx *rho, int n, const double *u_d, int k, const int *targets,
                        int nc, const int *controls, cplx *out)
{
    const uint64_t dim = (uint64_t)1 << n;
    cplx *col = (cplx *)malloc(sizeof(cplx) * dim);
    cplx *a = (cplx *)malloc(sizeof(cplx) * dim * dim);
    if (!col || !a) { free(col); free(a); return -1; }
    /* a = G rho */
    for (uint64_t c = 0; c < dim; ++c) {
        for (uint64_t r = 0; r < dim; ++r) col[r] = rho[r * dim + c];
        if (oracle_apply((double *)col, n, u_d, k, targets, nc, controls) != 0) {
            free(col); free(a); return -1;
        }
        for (uint64_t r = 0; r < dim; ++r) a[r * dim + c] = col[r];
    }
    /* out += (G a^dagger)^dagger = a G^dagger */
    for (uint64_t r = 0; r < dim; ++r) {
        for (uint64_t c = 0; c < dim; ++c) col[c] = conj(a[r * dim + c]);
        if (oracle_apply((double *)col, n, u_d, k, targets, nc, controls) != 0) {
            free(col); free(a); return -1;
        }
        for (uint64_t c = 0; c < dim; ++c) out[r * dim + c] += conj(col[c]);
    }
    free(col); free(a);
    return 0;
}

int oracle_dm_apply(double *rho_d, int n, const double *u_d, int k, const int *targets,
                    int nc, const int *controls)
{
    if (n < 1 || n > 12) return -1;
    const uint64_t dim = (uint64_t)1 << n;
    cplx *out = (cplx *)calloc(dim * dim, sizeof(cplx));
    if (!out) return -1;
    int rc = dm_conjugate((cplx *)rho_d, n, u_d, k, targets, nc, controls, out);
    if (rc == 0) memcpy(rho_d, out, sizeof(cplx) * dim * dim);
    free(out);
    return rc;
}

int oracle_dm_kraus(double *rho_d, int n, int nk, const double *kraus_d, int k,
                    const int *targets)
{
    if (n < 1 || n > 12 || nk < 1) return -1;
    const uint64_t dim = (uint64_t)1 << n;
    const size_t msz = (size_t)2 << (2 * k);   /* doubles per 2^k x 2^k complex matrix */
    cplx *out = (cplx *)calloc(dim * dim, sizeof(cplx));
    if (!out) return -1;
    int dummy = 0;
    for (int j = 0; j < nk; ++j)
        if (dm_conjugate((cplx *)rho_d, n, kraus_d + j * msz, k, targets, 0, &dummy, out) != 0) {
            free(out); return -1;
        }
    memcpy(rho_d, out, sizeof(cplx) * dim * dim);
    free(out);
    return 0;
}

/* Tr(rho P_t) for each Pauli string (X on xmask only, Z on zmask only, Y on
 * both): the sum over r, c of rho[r][c] P[c][r], P[c][r] the product of the
 * one-qubit entries.  Returns sum_t coeff_t Re Tr(rho P_t); imag_out gets the
 * imaginary part, term_out (if not NULL) each Tr(rho P_t). */
double oracle_dm_expectation(const double *rho_d, int n, int nterms, const uint64_t *xmask,
                             const uint64_t *zmask, const double *coeff, double *term_out,
                             double *imag_out)
{
    const cplx *rho = (const cplx *)rho_d;
    const uint64_t dim = (uint64_t)1 << n;
    double tot_re = 0.0, tot_im = 0.0;
    for (int t = 0; t < nterms; ++t) {
        cplx acc = 0;
        for (uint64_t r = 0; r < dim; ++r)
            for (uint64_t c = 0; c < dim; ++c) {
                cplx p = 1.0;
                for (int q = 0; q < n && p != 0; ++q) {
                    int code = (int)((xmask[t] >> q) & 1u) + 2 * (int)((zmask[t] >> q) & 1u);
                    p *= pauli_entry(code, bit_of(c, q), bit_of(r, q));
                }
                if (p != 0) acc += rho[r * dim + c] * p;
            }
        if (term_out) { term_out[2 * t] = creal(acc); term_out[2 * t + 1] = cimag(acc); }
        tot_re += coeff[t] * creal(acc);
        tot_im += coeff[t] * cimag(acc);
    }
    if (imag_out) *imag_out = tot_im;
    return tot_re;
}
