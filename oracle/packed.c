/*
 * ORACLE -- test infrastructure only.  Plain, slow, obviously correct FP64
 * reference for the packed-genotype operations of the GKL hot path.  Only the
 * test suite, the smoke check and the bench's CPU-baseline leg may load it; no
 * product code path calls it.  It shares no code with the GPU library.
 *
 * Storage format (reading of Section 1, where entries are 0, 1, 2 or missing):
 * SNP-major; column j in bytes [j*ld, j*ld + ld); individual i in byte
 * j*ld + i/4 at bits 2*(i%4); codes 0/1/2 are allele counts, 3 is missing.
 *
 * Standardised matrix (the paper leaves preprocessing unspecified, Table 2):
 *   A_ij = o_ij * (g_ij - mu_j) * s_j
 * with g = code for codes 0..2 and 0 for missing, o = [code != 3],
 * mu_j = c_j / nobs_j, s_j = 1 / sqrt(2 f_j (1 - f_j)), f_j = mu_j / 2
 * (binomial scaling), s_j = 0 for monomorphic or fully missing columns.
 * Missing entries are mean-imputed, so they contribute zero.
 */
#include <stdint.h>
#include <string.h>

static inline int code_at(const uint8_t* G, int64_t ld, int64_t i, int64_t j)
{
    return (G[j * ld + i / 4] >> (2 * (i % 4))) & 3;
}

/* Unpack to an n x p column-major int8 matrix; missing becomes -1. */
void oracle_decode(const uint8_t* G, int64_t n, int64_t p, int64_t ld, int8_t* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j)
        for (int64_t i = 0; i < n; ++i) {
            int c = code_at(G, ld, i, j);
            out[j * n + i] = (int8_t)(c == 3 ? -1 : c);
        }
}

/* Per-column counts of codes 1, 2 and 3 over the n real individuals. */
void oracle_counts(const uint8_t* G, int64_t n, int64_t p, int64_t ld,
                   int64_t* n1, int64_t* n2, int64_t* n3)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j) {
        int64_t a = 0, b = 0, c = 0;
        for (int64_t i = 0; i < n; ++i) {
            int k = code_at(G, ld, i, j);
            a += (k == 1);
            b += (k == 2);
            c += (k == 3);
        }
        n1[j] = a;
        n2[j] = b;
        n3[j] = c;
    }
}

static inline double entry(int c, double mu, double s)
{
    if (c == 3) return 0.0;              /* mean-imputed missing value */
    return ((double)c - mu) * s;
}

/* y = A v, summed over j in increasing order for each i. */
void oracle_matvec(const uint8_t* G, int64_t n, int64_t p, int64_t ld,
                   const double* mu, const double* s, const double* v, double* y)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i0 = 0; i0 < n; i0 += 256) {
        const int64_t i1 = i0 + 256 < n ? i0 + 256 : n;
        double acc[256];
        for (int64_t i = i0; i < i1; ++i) acc[i - i0] = 0.0;
        for (int64_t j = 0; j < p; ++j)
            for (int64_t i = i0; i < i1; ++i)
                acc[i - i0] += entry(code_at(G, ld, i, j), mu[j], s[j]) * v[j];
        for (int64_t i = i0; i < i1; ++i) y[i] = acc[i - i0];
    }
}

/* z = A^T u, summed over i in increasing order for each j. */
void oracle_rmatvec(const uint8_t* G, int64_t n, int64_t p, int64_t ld,
                    const double* mu, const double* s, const double* u, double* z)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i)
            acc += entry(code_at(G, ld, i, j), mu[j], s[j]) * u[i];
        z[j] = acc;
    }
}

/* Selected entries y_i = (A v)_i for a list of rows (sampled full-size checks). */
void oracle_matvec_rows(const uint8_t* G, int64_t n, int64_t p, int64_t ld,
                        const double* mu, const double* s, const double* v,
                        const int64_t* rows, int64_t nrows, double* y)
{
    (void)n;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        double acc = 0.0;
        const int64_t i = rows[r];
        for (int64_t j = 0; j < p; ++j) acc += entry(code_at(G, ld, i, j), mu[j], s[j]) * v[j];
        y[r] = acc;
    }
}

/* Selected entries z_j = (A^T u)_j for a list of columns. */
void oracle_rmatvec_cols(const uint8_t* G, int64_t n, int64_t p, int64_t ld,
                         const double* mu, const double* s, const double* u,
                         const int64_t* cols, int64_t ncols, double* z)
{
    (void)p;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < ncols; ++r) {
        double acc = 0.0;
        const int64_t j = cols[r];
        for (int64_t i = 0; i < n; ++i) acc += entry(code_at(G, ld, i, j), mu[j], s[j]) * u[i];
        z[r] = acc;
    }
}
