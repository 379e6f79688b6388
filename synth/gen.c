/*
 * Seeded synthetic genotype generator (bulk part).
 *
 * This file is input generation only: it draws genotypes and writes them in
 * the 2-bit packed, SNP-major storage format.  It holds none of the PCA
 * method's arithmetic (no standardisation, no products, no Lanczos).
 *
 * Model.  For individual i and SNP j the allele probability is
 *     P_ij = clip(base_j + sum_l A[i, l] * B[l, j], 0, 1)
 * which covers discrete subpopulations (A one-hot, B = per-population
 * frequency offsets), admixture (A = mixing weights) and planted low-rank
 * spikes.  The genotype is the number of successes in two Bernoulli(P_ij)
 * haplotype draws.  Haplotype 0 of individual i may be copied from another
 * individual (cryptic relatedness): it is then drawn with that individual's
 * uniform variate and probability.  With probability miss_rate the entry is
 * replaced by the missing code 3.
 *
 * Random numbers.  A counter-based generator: one 64-bit value per (j, i),
 * the SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014) applied
 * to a per-column key plus the individual index.  21 bits drive each
 * haplotype, 22 bits drive the missing-data draw.  Results do not depend on
 * the thread count.
 *
 * Packed format.  Column j occupies bytes [j*ld, j*ld + ld).  Individual i
 * sits in byte j*ld + i/4 at bits 2*(i%4) .. 2*(i%4)+1.  Codes 0/1/2 are
 * allele counts, 3 is missing.  Bits for i >= n and bytes beyond ceil(n/4)
 * are filled from pad_mode: 0..3 writes that code, -1 writes pseudo-random
 * garbage (used to prove consumers ignore padding).
 */
#include <stdint.h>
#include <string.h>

static inline uint64_t splitmix_out(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t column_key(uint64_t seed, int64_t j)
{
    return splitmix_out(splitmix_out(seed) + (uint64_t)j * 0xD1B54A32D192ED03ull);
}

static inline double prob_of(const double* base, const double* A, const double* B,
                             int64_t L, int64_t p, int64_t i, int64_t j)
{
    double P = base[j];
    for (int64_t l = 0; l < L; ++l) P += A[i * L + l] * B[l * p + j];
    if (P < 0.0) P = 0.0;
    if (P > 1.0) P = 1.0;
    return P;
}

#define U21(x) (((double)((x) & 0x1FFFFFull) + 0.5) * (1.0 / 2097152.0))

/* Columns j0 <= j < j1 of the p-column matrix into out (column j at
 * out + (j - j0) * ld).  Drawing a matrix in column ranges gives the same bytes
 * as drawing it at once.  Returns 0 on success, -1 on bad arguments. */
int synth_genotypes_range(int64_t n, int64_t p, int64_t j0, int64_t j1, int64_t ld,
                          uint64_t seed,
                          const double* base,      /* p */
                          int64_t L,
                          const double* A,         /* n x L row-major, may be NULL if L == 0 */
                          const double* B,         /* L x p row-major, may be NULL if L == 0 */
                          const int32_t* hap0_src, /* n, may be NULL (identity) */
                          double miss_rate,
                          int32_t pad_mode,
                          uint8_t* out)            /* (j1 - j0) * ld bytes */
{
    if (n <= 0 || p <= 0 || ld < (n + 3) / 4 || !base || !out) return -1;
    if (j0 < 0 || j1 > p || j0 >= j1) return -1;
    if (L > 0 && (!A || !B)) return -1;
    const int64_t nb = (n + 3) / 4;
    const uint64_t miss_thr = (uint64_t)(miss_rate * 4194304.0); /* 22-bit threshold */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = j0; j < j1; ++j) {
        const uint64_t key = column_key(seed, j);
        uint8_t* col = out + (j - j0) * ld;
        memset(col, 0, (size_t)ld);
        for (int64_t i = 0; i < n; ++i) {
            const uint64_t r = splitmix_out(key + (uint64_t)i);
            int code;
            if (((r >> 42) & 0x3FFFFFull) < miss_thr) {
                code = 3;
            } else {
                const double Pi = prob_of(base, A, B, L, p, i, j);
                int a1 = U21(r >> 21) < Pi;
                int a0;
                const int64_t src = hap0_src ? (int64_t)hap0_src[i] : i;
                if (src == i) {
                    a0 = U21(r) < Pi;
                } else {
                    const uint64_t rs = splitmix_out(key + (uint64_t)src);
                    a0 = U21(rs) < prob_of(base, A, B, L, p, src, j);
                }
                code = a0 + a1;
            }
            col[i >> 2] |= (uint8_t)(code << (2 * (i & 3)));
        }
        /* padding codes inside the last used byte, then padding bytes */
        for (int64_t i = n; i < nb * 4; ++i) {
            int c = pad_mode >= 0 ? (pad_mode & 3)
                                  : (int)(splitmix_out(key ^ 0xABCDEF12345ull ^ (uint64_t)i) & 3);
            col[i >> 2] |= (uint8_t)(c << (2 * (i & 3)));
        }
        for (int64_t b = nb; b < ld; ++b) {
            col[b] = pad_mode >= 0 ? (uint8_t)((pad_mode & 3) * 0x55)
                                   : (uint8_t)splitmix_out(key ^ 0x5A5A5A5Aull ^ (uint64_t)b);
        }
    }
    return 0;
}

/* The whole matrix (p * ld bytes). */
int synth_genotypes(int64_t n, int64_t p, int64_t ld, uint64_t seed, const double* base,
                    int64_t L, const double* A, const double* B, const int32_t* hap0_src,
                    double miss_rate, int32_t pad_mode, uint8_t* out)
{
    return synth_genotypes_range(n, p, 0, p, ld, seed, base, L, A, B, hap0_src, miss_rate,
                                 pad_mode, out);
}

/* Pack an explicit code matrix (n x p, column-major int8, values 0..3) into the
 * storage format above.  Used for hand-made fixtures. */
int synth_pack(int64_t n, int64_t p, int64_t ld, const int8_t* codes, int32_t pad_mode,
               uint8_t* out)
{
    if (n <= 0 || p <= 0 || ld < (n + 3) / 4 || !codes || !out) return -1;
    const int64_t nb = (n + 3) / 4;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j) {
        uint8_t* col = out + j * ld;
        memset(col, 0, (size_t)ld);
        for (int64_t i = 0; i < n; ++i)
            col[i >> 2] |= (uint8_t)((codes[j * n + i] & 3) << (2 * (i & 3)));
        const uint64_t key = column_key(0x7777ull, j);
        for (int64_t i = n; i < nb * 4; ++i) {
            int c = pad_mode >= 0 ? (pad_mode & 3) : (int)(splitmix_out(key + (uint64_t)i) & 3);
            col[i >> 2] |= (uint8_t)(c << (2 * (i & 3)));
        }
        for (int64_t b = nb; b < ld; ++b)
            col[b] = pad_mode >= 0 ? (uint8_t)((pad_mode & 3) * 0x55)
                                   : (uint8_t)splitmix_out(key ^ (uint64_t)b);
    }
    return 0;
}

/*
 * The random genotype model of the paper's Section 2 ("A simple model for
 * genomics data"), entry by entry so that large matrices can be drawn in
 * parallel.  Rows are individuals (i < n), columns SNPs (j < p).
 *   1. r rectangles [r0, r1] x [c0, c1] (inclusive) hold values v in {0, 1, 2};
 *      a later rectangle covers an earlier one; outside all of them the value
 *      is 0.
 *   2. nsignal positions drawn uniformly with replacement get random values in
 *      {0, 1, 2}, the last draw at a position holding.  Entry by entry this is:
 *      the entry is hit with probability q_hit = 1 - (1 - 1/(n p))^nsignal
 *      (passed in), and then takes a uniform value in {0, 1, 2}.
 *   3. Row i < n takes the values of row src[i] after step 2 (src[i] = i for
 *      rows that are not copies).
 * rect: r x 5 int64 (r0, r1, c0, c1, v).  Codes land in codes (column-major
 * n x p int8, when not NULL) and/or packed (p x ld, when not NULL).
 */
static inline int alg1_value(int64_t i, int64_t j, uint64_t key, const int64_t* rect, int64_t r,
                             uint64_t hit_thr)
{
    const uint64_t z = splitmix_out(key + (uint64_t)i);
    if ((z >> 11) < hit_thr) return (int)(((z & 0x1FFFFFull) * 3) >> 21);
    int v = 0;
    for (int64_t t = 0; t < r; ++t) {
        const int64_t* R = rect + 5 * t;
        if (i >= R[0] && i <= R[1] && j >= R[2] && j <= R[3]) v = (int)R[4];
    }
    return v;
}

int synth_algorithm1(int64_t n, int64_t p, int64_t r, const int64_t* rect, double q_hit,
                     const int32_t* src, uint64_t seed, int8_t* codes, int64_t ld,
                     uint8_t* packed)
{
    if (n <= 0 || p <= 0 || r < 0 || (r > 0 && !rect) || !src) return -1;
    if (packed && ld < (n + 3) / 4) return -1;
    const uint64_t hit_thr = (uint64_t)(q_hit * 9007199254740992.0);   /* 53-bit threshold */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < p; ++j) {
        const uint64_t key = column_key(seed, j);
        uint8_t* col = packed ? packed + j * ld : NULL;
        if (col) memset(col, 0, (size_t)ld);
        for (int64_t i = 0; i < n; ++i) {
            const int c = alg1_value(src[i], j, key, rect, r, hit_thr);
            if (codes) codes[j * n + i] = (int8_t)c;
            if (col) col[i >> 2] |= (uint8_t)(c << (2 * (i & 3)));
        }
    }
    return 0;
}
