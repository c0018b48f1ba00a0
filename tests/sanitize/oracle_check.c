/* Drives every entry point of the oracle (oracle/qsv_oracle.c) on small
 * seeded inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: any out-of-bounds access, leak or undefined
 * operation aborts the run.  Also checks a few invariants on the way (norm
 * kept by unitaries, probabilities summing to one, serial and threaded
 * gates agreeing).  Prints "ok" and returns 0. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_set_threads(int t);
int oracle_apply(double *psi, int n, const double *u, int k, const int *targets, int nc,
                 const int *controls);
void oracle_probs(const double *psi, int n, double *out);
double oracle_prob_bits(const double *psi, int n, int m, const int *qubits, const int *bits);
double oracle_expectation(const double *psi, int n, int nterms, const uint64_t *xmask,
                          const uint64_t *zmask, const double *coeff, double *term_out,
                          double *imag_out);
int oracle_measure(double *psi, int n, int q, double u, double *probs_out);
int oracle_sample(const double *psi, int n, int shots, const double *u, uint64_t *out);
int oracle_dealloc(const double *psi, int n, int q, double tau, double *out);
int oracle_apply_math(double *psi, int n, int w, const int *qubits, const uint32_t *table, int nc,
                      const int *controls);
int oracle_dm_apply(double *rho, int n, const double *u, int k, const int *targets, int nc,
                    const int *controls);
int oracle_dm_kraus(double *rho, int n, int nk, const double *kraus, int k, const int *targets);
double oracle_dm_expectation(const double *rho, int n, int nterms, const uint64_t *xmask,
                             const uint64_t *zmask, const double *coeff, double *term_out,
                             double *imag_out);

static uint64_t rs = 0x9e3779b97f4a7c15ull;
static double urand(void) {
    rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;
    return (double)(rs >> 11) / 9007199254740992.0;
}

/* a random unitary of size d (Gram-Schmidt on random complex columns),
 * interleaved re/im, row-major */
static void rand_unitary(double *u, int d) {
    for (int i = 0; i < 2 * d * d; ++i) u[i] = urand() - 0.5;
    for (int c = 0; c < d; ++c) {
        for (int p = 0; p < c; ++p) {
            double re = 0, im = 0;   /* <col p, col c> */
            for (int r = 0; r < d; ++r) {
                const double *a = u + 2 * (r * d + p), *b = u + 2 * (r * d + c);
                re += a[0] * b[0] + a[1] * b[1];
                im += a[0] * b[1] - a[1] * b[0];
            }
            for (int r = 0; r < d; ++r) {
                const double *a = u + 2 * (r * d + p);
                double *b = u + 2 * (r * d + c);
                b[0] -= re * a[0] - im * a[1];
                b[1] -= re * a[1] + im * a[0];
            }
        }
        double nn = 0;
        for (int r = 0; r < d; ++r) nn += u[2 * (r * d + c)] * u[2 * (r * d + c)] + u[2 * (r * d + c) + 1] * u[2 * (r * d + c) + 1];
        nn = sqrt(nn);
        for (int r = 0; r < d; ++r) { u[2 * (r * d + c)] /= nn; u[2 * (r * d + c) + 1] /= nn; }
    }
}

static double norm2(const double *psi, uint64_t dim) {
    double s = 0;
    for (uint64_t i = 0; i < 2 * dim; ++i) s += psi[i] * psi[i];
    return s;
}

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)

int main(void) {
    const int n = 9;
    const uint64_t dim = 1ull << n;
    double *psi = calloc(2 * dim, sizeof(double));
    double *psi2 = calloc(2 * dim, sizeof(double));
    psi[0] = 1.0;
    double u[2 * 32 * 32];
    for (int g = 0; g < 60; ++g) {
        const int k = 1 + g % 4, nc = g % 3;
        int q[9];
        for (int i = 0; i < n; ++i) q[i] = i;
        for (int i = n - 1; i > 0; --i) { int j = (int)(urand() * (i + 1)); int t = q[i]; q[i] = q[j]; q[j] = t; }
        rand_unitary(u, 1 << k);
        memcpy(psi2, psi, 2 * dim * sizeof(double));
        CHECK(oracle_apply(psi, n, u, k, q, nc, q + k) == 0);
        oracle_set_threads(3);
        CHECK(oracle_apply(psi2, n, u, k, q, nc, q + k) == 0);
        oracle_set_threads(1);
        CHECK(memcmp(psi, psi2, 2 * dim * sizeof(double)) == 0);
        CHECK(fabs(norm2(psi, dim) - 1.0) < 1e-12);
    }
    CHECK(oracle_apply(psi, n, u, 0, NULL, 0, NULL) == -1);
    double *p = calloc(dim, sizeof(double));
    oracle_probs(psi, n, p);
    double tot = 0;
    for (uint64_t i = 0; i < dim; ++i) tot += p[i];
    CHECK(fabs(tot - 1.0) < 1e-12);
    int qs[3] = {1, 4, 7}, bits[3] = {1, 0, 1};
    const double pb = oracle_prob_bits(psi, n, 3, qs, bits);
    CHECK(pb >= 0.0 && pb <= 1.0);
    uint64_t xm[4] = {0x3, 0x0, 0x101, 0x1f0}, zm[4] = {0x0, 0x1c, 0x101, 0x0f};
    double coeff[4] = {0.5, -1.0, 0.25, 2.0}, terms[8], imag = 0;
    const double e = oracle_expectation(psi, n, 4, xm, zm, coeff, terms, &imag);
    CHECK(isfinite(e) && fabs(imag) < 1e-12);
    double uu[16];
    for (int i = 0; i < 16; ++i) uu[i] = urand();
    uint64_t samples[16];
    CHECK(oracle_sample(psi, n, 16, uu, samples) == 0);
    for (int i = 0; i < 16; ++i) CHECK(samples[i] < dim);
    double probs[2];
    CHECK(oracle_measure(psi, n, 3, 0.3, probs) >= 0);
    CHECK(fabs(norm2(psi, dim) - 1.0) < 1e-12);
    double *out = calloc(dim, sizeof(double));
    const int r = oracle_dealloc(psi, n, 3, 1e-12, out);   /* qubit 3 was just measured */
    CHECK(r == 0 || r == 1);
    uint32_t table[16];
    for (uint32_t x = 0; x < 16; ++x) table[x] = (x * 7 + 3) & 15;
    int mq[4] = {0, 2, 5, 6}, mc[1] = {8};
    CHECK(oracle_apply_math(psi, n, 4, mq, table, 1, mc) == 0);
    CHECK(fabs(norm2(psi, dim) - 1.0) < 1e-12);
    /* density matrix of 4 qubits */
    const int dn = 4;
    const uint64_t dd = 1ull << (2 * dn);
    double *rho = calloc(2 * dd, sizeof(double));
    rho[0] = 1.0;
    for (int g = 0; g < 10; ++g) {
        int t[2] = {g % dn, (g + 1) % dn}, c[1] = {(g + 2) % dn};
        rand_unitary(u, 4);
        CHECK(oracle_dm_apply(rho, dn, u, 2, t, g % 2, c) == 0);
    }
    double kr[2 * 2 * 4];   /* amplitude damping, gamma 0.3 */
    memset(kr, 0, sizeof kr);
    kr[0] = 1.0; kr[6] = sqrt(0.7);
    kr[8 + 2] = sqrt(0.3);
    int kt[1] = {2};
    CHECK(oracle_dm_kraus(rho, dn, 2, kr, 1, kt) == 0);
    double tr = 0;
    for (uint64_t i = 0; i < (1ull << dn); ++i) tr += rho[2 * (i * (1ull << dn) + i)];
    CHECK(fabs(tr - 1.0) < 1e-12);
    const double de = oracle_dm_expectation(rho, dn, 4, xm, zm, coeff, terms, &imag);
    CHECK(isfinite(de));
    free(psi); free(psi2); free(p); free(out); free(rho);
    printf("ok\n");
    return 0;
}
