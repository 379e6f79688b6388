/*
 * gkl.h -- C ABI of the MI355X (gfx950) Golub-Kahan-Lanczos library for the
 * top-k principal components of a 2-bit packed genotype matrix.
 *
 * Method: Chen, Noack & Edelman, "Fast computation of the principal components
 * of genotype matrices in Julia", arXiv:1808.03374.
 *   - Section 3 (Golub-Kahan-Lanczos bidiagonalization): A V_j = U_j B_j with
 *     B_j upper bidiagonal; top singular triplets from the SVD of B_j.
 *   - Section 3 "Thick restarting": restart from the leading ordinary Ritz
 *     vectors to bound memory and roundoff.
 *   - Section 3 "Choice of reorthogonalization strategy": full
 *     reorthogonalization by doubly reorthogonalized classical Gram-Schmidt
 *     (CGS2), optionally with an adaptive second pass; or partial
 *     reorthogonalization (PRO) with threshold omega (1e-8 in the experiments).
 *   - Section 3 "Convergence criteria": |sigma - sigma~_i| <= beta_j |P_{j,i}|.
 *   - Section 5 (conclusions): block Lanczos as the BLAS3 extension, here the
 *     mixed-precision blocked variant.
 *
 * Plain C99. No C++ types cross the ABI, no exception escapes, every fallible
 * entry point returns a gkl_status and leaves a message in gkl_last_error().
 *
 * Matrix and storage format
 *   G is n individuals x p SNPs.  Storage is SNP-major: column j occupies bytes
 *   [j*ld, j*ld + ld) with ld >= ceil(n/4); individual i sits in byte
 *   j*ld + i/4 at bits 2*(i%4)..2*(i%4)+1.  Codes 0/1/2 are allele counts and
 *   3 is missing.  Bits for i >= n and bytes beyond ceil(n/4) are ignored.
 *   The operator is the standardized matrix with mean imputation
 *       A_ij = o_ij * (g_ij - mu_j) * s_j,
 *   g = code (0 for missing), o = [code != 3], mu_j = c_j / nobs_j with
 *   c_j = n1_j + 2 n2_j and nobs_j = n - n3_j, s_j = 1/sqrt(mu_j (1 - mu_j/2))
 *   (binomial scaling), s_j = 0 when nobs_j = 0 or the column is monomorphic.
 *
 * Pointers
 *   Unless stated otherwise every array argument is a DEVICE pointer on the
 *   current HIP device (for example torch.Tensor.data_ptr() on ROCm).  Output
 *   arrays are caller-allocated, column-major, FP64.  G is borrowed: it must
 *   stay valid and unchanged until gkl_destroy.  Contexts are not thread-safe;
 *   use one context per thread.
 *
 * Streams
 *   All device work of a context runs on options.stream (NULL = the default
 *   stream).  Every entry point returns after its outputs are written, i.e. it
 *   is synchronous with respect to the host.
 */
#ifndef GKL_H
#define GKL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gkl_ctx gkl_ctx;

typedef enum gkl_status {
    GKL_OK = 0,
    GKL_ERR_INVALID = 1,      /* bad argument; nothing was changed */
    GKL_ERR_NOMEM = 2,        /* device allocation failed */
    GKL_ERR_DEVICE = 3,       /* a HIP call or kernel launch failed */
    GKL_NOT_CONVERGED = 4,    /* max_matvecs reached or the basis (max_steps) filled
                                 without restart; best Ritz triplets written */
    GKL_ERR_BREAKDOWN = 5,    /* no new direction could be found */
    GKL_ERR_INTERNAL = 6,
    GKL_ERR_UNSUPPORTED = 7   /* option combination not built */
} gkl_status;

/* GKL_REORTH_FULL: CGS2 of every new vector against its whole basis.
 * GKL_REORTH_PARTIAL: CGS2 only when the estimated loss of orthogonality (PRO
 * recurrences) exceeds options.pro_omega.
 * GKL_REORTH_ONESIDED: CGS2 on the shorter side only (U when n <= p, else V);
 * each new long-side vector is only checked against its basis (one projection
 * instead of CGS2's three passes) until an overlap exceeds min(pro_omega, tol)
 * times its norm, from which step on both sides are reorthogonalised; the
 * returned long-side vectors are recomputed from the short side
 * (v_i = A^T u_i / ||A^T u_i|| when n <= p).
 * Section 3, "Choice of reorthogonalization strategy"; FP64 path only. */
enum gkl_reorth { GKL_REORTH_FULL = 0, GKL_REORTH_PARTIAL = 1, GKL_REORTH_ONESIDED = 2 };
/* GKL_PREC_FP64: single-vector FP64 GKL.  GKL_PREC_MIXED: blocked GKL whose two
 * products run on the matrix cores with split-BF16 vector tiles (hi + lo, FP32
 * accumulation per K chunk, FP64 across chunks); every other quantity FP64.
 * GKL_PREC_MIXED_INT8: the same blocked GKL with the products on the int8
 * matrix cores: the vector block is rounded per column to 22-bit integers
 * (power-of-two column scale) in three 8-bit limbs and accumulated exactly in
 * int32, so the products' only rounding is that quantisation.
 * GKL_PREC_BLOCK_FP64: the same blocked GKL with FP64-accurate block products:
 * each column is rounded to a 52-bit integer of a power-of-two scale and split
 * into seven 8-bit limbs (as GKL_FP64_LIMBS); two columns share one pass over
 * the matrix (their 14 limb columns fill one 16-column MFMA tile), so a block of
 * b vectors costs ceil(b/2) passes. */
enum gkl_precision {
    GKL_PREC_FP64 = 0, GKL_PREC_MIXED = 1, GKL_PREC_MIXED_INT8 = 2, GKL_PREC_BLOCK_FP64 = 3
};
/* How a GKL_PREC_FP64 context forms its products A v and A^T u (Section 3: one
 * of each per Lanczos step).  Both are FP64-accurate and pass the same parity
 * tests.  GKL_FP64_LUT: 256-entry FP64 tables per four genotypes in LDS, one
 * table read and one FP64 add per byte.  GKL_FP64_LIMBS: the int8 matrix cores
 * with the vector scaled by a power of two at least its largest magnitude,
 * rounded to a 52-bit integer and split into seven 8-bit limbs; the limb sums
 * are exact and recombined in FP64, so the product carries the vector's
 * quantisation (at most 2^-53 of that scale per entry) and FP64 roundings only.
 * GKL_FP64_LUT_LIMBS: tables for A v, limbs for A^T u.  GKL_FP64_AUTO: LIMBS
 * when n p >= 1e9 (250 MB packed), else LUT.  Measured at 50,000 x 500,000: A v
 * 1.13 ms in limbs against 1.29 ms from the tables, A^T u 1.14 ms against 2.09
 * ms; at 10,000 x 100,000 a 720-product solve takes 94 ms in limbs and 97 ms
 * from the tables, and below that the tables avoid the two small quantisation
 * kernels each limb product adds. */
enum gkl_fp64_products {
    GKL_FP64_AUTO = 0, GKL_FP64_LUT = 1, GKL_FP64_LIMBS = 2, GKL_FP64_LUT_LIMBS = 3
};

/* Thick restart (Section 3, "Thick restarting"), used when krylov_dim > 0.
 * GKL_RESTART_RITZ: keep the l leading ordinary Ritz vectors (Wu & Simon); the
 * projected matrix restarts as diag(sigma) with one coupling column.
 * GKL_RESTART_HARMONIC: keep the l leading harmonic Ritz vectors of A^T A on
 * span(V_m) (Baglama & Reichel, SIAM J. Sci. Comput. 27, 2005): the squared
 * singular values of [B_m, beta_m e_m], vectors V_m B_m^-1 p_j, and the
 * direction their residuals share; the projected matrix restarts with a dense
 * l x l head.  Convergence tests and the returned triplets use ordinary Ritz
 * values either way.  Built for GKL_PREC_FP64 with GKL_REORTH_FULL (the
 * partial reorthogonalisation recurrences assume the diagonal head); a restart
 * whose basis recorded a breakdown (a zero recurrence scalar, B_m singular)
 * falls back to the ordinary kind. */
enum gkl_restart { GKL_RESTART_RITZ = 0, GKL_RESTART_HARMONIC = 1 };

/* Options.  Always initialise with gkl_options_default(). */
typedef struct gkl_options {
    uint32_t struct_size;     /* sizeof(gkl_options), set by gkl_options_default */
    int32_t krylov_dim;       /* m, vectors kept before a thick restart; 0 = no restart
                                 (FP64), or max(128, 3k + b) rounded to b (blocked) */
    int32_t keep;             /* l, Ritz vectors kept at a restart; 0 = k + (m - k)/2
                                 (FP64) or k + (m - k)/4 (blocked) */
    int32_t precision;        /* gkl_precision */
    int32_t block_width;      /* b of the mixed blocked variant (1..32); 0 = 8 */
    int32_t adaptive_cgs2;    /* 1: second Gram-Schmidt pass only when the first pass
                                 shrank the vector below 1/sqrt(2) of its norm */
    int32_t check_every;      /* steps between convergence tests; 0 = auto (when the
                                 basis is full if restarting; else every 5 steps up
                                 to a 20-vector basis, then each time it has grown
                                 by a quarter, as the projected SVD costs O(j^3);
                                 blocked with the default basis and n p >= 4e9:
                                 also before the first restart, from k + b columns
                                 on each time the basis has grown by a quarter) */
    int32_t max_steps;        /* cap on the basis size without restart; 0 = min(512,
                                 min(n, p)).  A solve without restart that fills the
                                 basis before converging returns GKL_NOT_CONVERGED. */
    double pro_omega;         /* PRO threshold on the orthogonality estimate; 0 = 1e-8 */
    int64_t max_matvecs;      /* stop with GKL_NOT_CONVERGED after this many; 0 = unlimited */
    uint64_t seed;            /* start vector seed when v0 is NULL */
    const double* v0;         /* optional device start vector (p values; p*b when blocked) */
    int64_t ld_bytes;         /* bytes per SNP column of G; 0 = ceil(n/4) */
    void* stream;             /* hipStream_t; NULL = default stream */
    int32_t trace;            /* 1: record a per-step trace (gkl_get_trace) */
    int32_t verbose;          /* 1: progress lines on stderr */
    int32_t timing;           /* t > 0: bracket the first of every t product launches
                                 (1 = every launch) with HIP events and report the
                                 product kernel time in gkl_info; each bracket
                                 costs the stream a few microseconds */
    int32_t autotune;         /* batched: 1 = time candidate product geometries at
                                 create and keep the fastest; 0 = fixed geometry */
    int32_t graph;            /* batched: 1 (default) = each Lanczos step is one HIP
                                 graph launch; 0 = the same kernels launched one by one */
    int32_t fp64_products;    /* gkl_fp64_products (GKL_PREC_FP64 contexts; the
                                 batched path forms A v from the tables in every case
                                 and A^T u in limbs for _LIMBS, _LUT_LIMBS, and for
                                 _AUTO from 1 GB of packed genotypes in the batch) */
    int32_t restart;          /* gkl_restart; 0 = GKL_RESTART_RITZ */
} gkl_options;

/* Run statistics (host struct). */
typedef struct gkl_info {
    int64_t matvecs;          /* products A v or A^T u; a block product counts b */
    int64_t passes_over_G;    /* times the packed matrix was streamed */
    int64_t steps;            /* Lanczos steps (block steps in the blocked variant) */
    int64_t restarts;
    int64_t reorths;          /* Gram-Schmidt reorthogonalizations performed */
    int32_t nconv;            /* leading Ritz values meeting the tolerance */
    int32_t converged;        /* 1 when all k met the tolerance */
    double sum_residual_est;  /* sum_i beta_j |P_{j,i}| over the k returned values */
    double max_residual_rel;  /* max_i residual_i / sigma_1 */
    double solve_ms;
    double create_ms;
    double matvec_kernel_ms;  /* with options.timing: summed A v kernel time */
    double rmatvec_kernel_ms; /* with options.timing: summed A^T u kernel time */
    int64_t timed_matvecs;    /* launches behind matvec_kernel_ms */
    int64_t timed_rmatvecs;   /* launches behind rmatvec_kernel_ms */
    double matvec_core_ms;    /* with options.timing: the same launches, main kernel
                                 only (a blocked product is several kernels: vector
                                 split, column sums, the matrix-core kernel, reduce);
                                 equal to matvec_kernel_ms on the FP64 path */
    double rmatvec_core_ms;   /* likewise for the A^T u / A^T X products */
    int32_t fp64_products;    /* format the FP64 products ran in: GKL_FP64_LUT,
                                 _LIMBS or _LUT_LIMBS (0 on the blocked and LOCO
                                 paths) */
    int32_t reserved;
} gkl_info;

void gkl_options_default(gkl_options* opt);
const char* gkl_status_string(gkl_status s);
/* Last error message of ctx; ctx == NULL gives the calling thread's last
 * message from gkl_create / gkl_create_ex / gkl_create_batched. */
const char* gkl_last_error(const gkl_ctx* ctx);

/*
 * gkl_create / gkl_create_ex
 *   Validate the arguments, compute the column statistics (counts, mu, s) on the
 *   device and allocate the solver workspace for a top-k solve (the paper's
 *   preprocessing, whose content it leaves open: Section 4, Table 2 gives its
 *   time only; the standardisation above is this library's reading).  An FP64
 *   context builds one internal copy of G per product in the format that
 *   options.fp64_products selects (about n p / 4 bytes each), a blocked one
 *   (GKL_PREC_MIXED*) the two layouts of its matrix-core products.
 *   G      device, p*ld bytes, SNP-major 2-bit codes (see above), borrowed.
 *   n, p   individuals and SNPs, both >= 1.
 *   k      singular triplets wanted, 1 <= k <= min(n, p).
 *   tol    relative tolerance: stop when beta_j |P_{j,i}| <= tol * sigma~_1 for
 *          every i < k; must be > 0.
 *   reorth gkl_reorth.
 *   out    receives the context; unchanged on failure.
 *   Errors: GKL_ERR_INVALID (n, p < 1; k out of range; tol <= 0; m != 0 and
 *   m <= k; ld < ceil(n/4); NULL G or out; bad option values), GKL_ERR_NOMEM,
 *   GKL_ERR_DEVICE.  On any error nothing is allocated.
 */
gkl_status gkl_create(const uint8_t* G, int64_t n, int64_t p, int32_t k, double tol,
                      int32_t reorth, gkl_ctx** out);
gkl_status gkl_create_ex(const uint8_t* G, int64_t n, int64_t p, int32_t k, double tol,
                         int32_t reorth, const gkl_options* opt, gkl_ctx** out);

/*
 * gkl_solve
 *   Run the Lanczos iteration and write the top-k triplets (Section 3: GKL
 *   bidiagonalisation, thick restart, CGS2 or partial reorthogonalisation, the
 *   convergence test beta_j |P_{j,i}| <= tol sigma~_1; blocked: Section 5).
 *   sigma  device, k values, descending.
 *   U      device, n x k column-major with leading dimension ldu >= n (scores).
 *   V      device, p x k column-major with leading dimension ldv >= p (loadings).
 *   info   host, may be NULL.
 *   Sign rule: the largest-magnitude entry of each V column is positive
 *   (lowest index on ties); the U column is flipped with it.
 *   Returns GKL_NOT_CONVERGED (outputs still written) when max_matvecs ran out.
 *   A context can be solved repeatedly; each solve starts from the start vector.
 */
gkl_status gkl_solve(gkl_ctx* ctx, double* sigma, double* U, int64_t ldu, double* V,
                     int64_t ldv, gkl_info* info);

/* Release everything owned by ctx.  NULL-safe. */
void gkl_destroy(gkl_ctx* ctx);

/*
 * Batched solves of many uneven matrices (per-chromosome PCAs), each problem
 * by the FP64 GKL iteration of Section 3.
 *   count     number of problems (1..1024).
 *   G, n, p   host arrays of count device pointers / sizes; each problem as above.
 *   The context solves all problems together: every Lanczos half-step of all
 *   still-running problems is one persistent kernel launch, and problems drop
 *   out as they converge.  Options apply to every problem (FP64, full reorth).
 */
gkl_status gkl_create_batched(int32_t count, const uint8_t* const* G, const int64_t* n,
                              const int64_t* p, int32_t k, double tol, int32_t reorth,
                              const gkl_options* opt, gkl_ctx** out);
/*   sigma, U, V: host arrays of count device pointers; ldu, ldv host arrays.
 *   infos: host array of count gkl_info, may be NULL. */
gkl_status gkl_solve_batched(gkl_ctx* ctx, double* const* sigma, double* const* U,
                             const int64_t* ldu, double* const* V, const int64_t* ldv,
                             gkl_info* infos);
/*   Product geometry of a batched context (after autotuning when options.autotune
 *   was set): K-split target in workgroups per problem and persistent grid size
 *   of the A v and A^T u launches, and their measured launch times in ms (0 when
 *   not tuned).  Any pointer may be NULL. */
gkl_status gkl_batched_plan(const gkl_ctx* ctx, int64_t* mv_target, int64_t* rmv_target,
                            int32_t* grid_mv, int32_t* grid_rmv, double* mv_ms, double* rmv_ms);

/*
 * gkl_create_loco -- leave-one-block-out PCAs (one per chromosome, say): for
 * every contiguous SNP block q = [block_start[q], block_start[q+1]) of the
 * n x p matrix G, the top-k triplets of G without that block, all solved
 * together.  Problem q runs the GKL iteration of Section 3 (full CGS2, thick
 * restart when krylov_dim > 0) with its right vectors in the whole p-space and
 * zero on its own block; the products of all problems are then one block
 * product with the whole matrix per half-step (nblocks columns, on the matrix
 * cores: options.precision must be GKL_PREC_MIXED or GKL_PREC_MIXED_INT8),
 * so the matrix is streamed once per step for all problems instead of
 * nblocks - 1 times.  Column statistics are those of the whole matrix.
 *   G           device, SNP-major 2-bit codes as for gkl_create, borrowed.
 *   nblocks     2..32;  block_start  host array of nblocks + 1 increasing
 *               offsets, block_start[0] = 0 and block_start[nblocks] = p.
 *   k           1 <= k <= min(n, p - largest block).
 * Solve with gkl_solve_batched (count = nblocks): V of problem q is p x k with
 * zeros on block q's rows; options.v0 holds nblocks p-vectors back to back.
 * Errors: GKL_ERR_INVALID (arguments), GKL_ERR_UNSUPPORTED (FP64 precision),
 * GKL_ERR_NOMEM, GKL_ERR_DEVICE.
 */
gkl_status gkl_create_loco(const uint8_t* G, int64_t n, int64_t p, int32_t nblocks,
                           const int64_t* block_start, int32_t k, double tol,
                           const gkl_options* opt, gkl_ctx** out);

/* ---------------- kernel-level entry points on an existing context ----------
 * Used by the parity tests and the bench; same conventions as above.  All
 * pointers are device pointers; every call is synchronous.  A batched context
 * is rejected with GKL_ERR_INVALID by all of them. */

/* Column statistics of the context's matrix (the preprocessing read above):
 * count (int64, p: n1 + 2 n2), nobs (int64, p: n - n3), mean (p), inv_sd (p).
 * Any context kind; any pointer may be NULL to skip it. */
gkl_status gkl_column_stats(gkl_ctx* ctx, int64_t* count, int64_t* nobs, double* mean,
                            double* inv_sd);
/* Decode the caller's G (the storage format above; the paper's entries 0, 1, 2
 * or missing, Section 1) to an n x p column-major int8 matrix, missing = -1.
 * Any context kind (it reads G, which the context borrows). */
gkl_status gkl_unpack(gkl_ctx* ctx, int8_t* out);
/* y = A v (v: p values, y: n values) in FP64: the product every Lanczos step
 * applies (Section 3), in the context's options.fp64_products format.  Needs a
 * GKL_PREC_FP64 context (its product layouts); a blocked context gives
 * GKL_ERR_INVALID. */
gkl_status gkl_matvec(gkl_ctx* ctx, const double* v, double* y);
/* z = A^T u (u: n values, z: p values) in FP64; GKL_PREC_FP64 context only. */
gkl_status gkl_rmatvec(gkl_ctx* ctx, const double* u, double* z);
/* Y = A W for b columns, 1 <= b <= 32 (W: p x b, Y: n x b, column-major,
 * leading dims p and n): the block product of the blocked variant (block
 * Lanczos, Section 5), through the matrix-core path of the context's precision
 * (GKL_PREC_MIXED: W split into bf16 hi + lo, FP32 accumulate per K-chunk, FP64
 * across chunks; GKL_PREC_MIXED_INT8: W in exact int8 limbs of a 22-bit
 * per-column fixed point, int32 accumulation; GKL_PREC_BLOCK_FP64: seven limbs
 * of a 52-bit fixed point, FP64-accurate, one pass per pair of columns), with
 * FP64 centring and missing-value terms.  Needs a blocked context; an FP64 one
 * gives GKL_ERR_INVALID. */
gkl_status gkl_matmat_mixed(gkl_ctx* ctx, const double* W, int32_t b, double* Y);
/* Z = A^T X for b columns (X: n x b, Z: p x b), the same matrix-core path and
 * the same requirements. */
gkl_status gkl_rmatmat_mixed(gkl_ctx* ctx, const double* X, int32_t b, double* Z);
/* Per-step trace of the last solve (options.trace = 1), as rows of
 * GKL_TRACE_FIELDS doubles: step, alpha, beta (the bidiagonal's entries of
 * Section 3), reorth_left, reorth_right, restart, max_residual_rel.
 * buf is HOST memory of cap doubles; *written receives the number of rows. */
#define GKL_TRACE_FIELDS 7
gkl_status gkl_get_trace(gkl_ctx* ctx, double* buf, int64_t cap, int64_t* written);

/*
 * gkl_dense_svd -- the small dense SVD used for Ritz extraction (Section 3,
 * "Convergence criteria": the top Ritz values and the residual bound come from
 * the SVD of the projected matrix B), exposed for testing:
 * B (m x m, column-major, device) = P diag(S) Q^T with S descending.
 * 1 <= m <= 1024.  m <= 96: one workgroup with everything in LDS;
 * 96 < m <= 128: the matrix in LDS and the rotations logged to a device buffer
 * (5.2 MB at m = 128) and replayed; m > 128: working matrices in device memory,
 * each round of a sweep one launch spread over workgroups, the host reading a
 * rotation flag after each sweep.  The buffer of the last two cases is
 * allocated and freed inside the call.
 * P, Q: m x m column-major device; S: m device.  stream may be NULL.
 * Errors: GKL_ERR_INVALID (NULL pointer, m out of range), GKL_ERR_NOMEM /
 * GKL_ERR_DEVICE.
 */
gkl_status gkl_dense_svd(const double* B, int32_t m, double* P, double* S, double* Q,
                         void* stream);

/*
 * gkl_dense_svd_noalloc -- gkl_dense_svd for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and the same result bit for bit, for
 * 1 <= m <= GKL_DENSE_SVD_NOALLOC_MAX_M; larger m returns GKL_ERR_INVALID.
 * It calls no allocating routine: the rotation log / working matrices live in
 * a fixed 5 MiB device array inside the library, one copy per GPU, held until
 * the process ends.  All calls on one GPU share that array, so calls that
 * overlap in time on one GPU (several streams or host threads) race; serialise
 * them.  The call is synchronous on `stream` (for m > 128 it also waits on
 * the stream once per sweep), so it cannot itself be captured into a graph.
 */
#define GKL_DENSE_SVD_NOALLOC_MAX_M 256
gkl_status gkl_dense_svd_noalloc(const double* B, int32_t m, double* P, double* S, double* Q,
                                 void* stream);

/*
 * gkl_read_rate -- diagnostic, not part of the method: the time of a plain
 * streaming read of `bytes` bytes of device memory at buf (each workgroup reads
 * one contiguous megabyte in 16-byte loads; nothing is written), averaged over
 * `reps` launches on `stream` (NULL = default) after one untimed launch.  It
 * measures the read rate this GPU achieves in practice, the ceiling against
 * which the product kernels, which stream the packed matrix once per product,
 * are judged.  buf must be 16-byte aligned; bytes >= 16 (a tail that is not a
 * multiple of 16 is not read).  *ms_per_read (host) receives milliseconds.
 * Errors: GKL_ERR_INVALID (NULL pointer, misaligned buf, bytes < 16,
 * reps < 1), GKL_ERR_DEVICE.
 */
gkl_status gkl_read_rate(const void* buf, int64_t bytes, int32_t reps, void* stream,
                         double* ms_per_read);

#ifdef __cplusplus
}
#endif

#endif /* GKL_H */
