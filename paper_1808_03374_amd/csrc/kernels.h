// Kernel launch interface used by the host engine (internal).
#pragma once

#include "common.h"

namespace gkl {

// Column statistics, device arrays of length p.
struct ColStats {
    int64_t* count;   // c_j = n1 + 2 n2
    int64_t* nobs;    // n - n3
    int64_t* n3;      // missing count
    double* mean;     // mu_j
    double* inv_sd;   // s_j
};

// Counts of codes 1, 2, 3 in one 32-bit word holding 16 codes; `valid` low codes
// are real individuals (the rest is padding and ignored).
__device__ __forceinline__ void count_word(uint32_t w, int valid, int64_t& c1, int64_t& c2,
                                           int64_t& c3)
{
    const uint32_t keep = valid >= 16 ? 0xFFFFFFFFu : ((1u << (2 * valid)) - 1u);
    w &= keep;
    const uint32_t lo = w & 0x55555555u;
    const uint32_t hi = (w >> 1) & 0x55555555u;
    c1 += __popc(lo & ~hi);
    c2 += __popc(hi & ~lo);
    c3 += __popc(lo & hi);
}

// Column j's statistics from its exact code counts: mean = (n1 + 2 n2) / nobs
// and scale 1/sqrt(2 f (1 - f)) with f = mean/2, in one fixed order of correctly
// rounded operations (every kernel that forms them calls this).
__device__ __forceinline__ void store_colstats(const ColStats& st, int64_t j, int64_t n,
                                               int64_t c1, int64_t c2, int64_t c3)
{
#pragma clang fp contract(off)
    const int64_t nobs = n - c3;
    const int64_t cnt = c1 + 2 * c2;
    double mu = 0.0, s = 0.0;
    if (nobs > 0) {
        mu = (double)cnt / (double)nobs;
        const double f = 0.5 * mu;
        const double t = 1.0 - f;
        const double var = mu * t;
        if (var > 0.0) {
            const double d = sqrt(var);
            s = 1.0 / d;
        }
    }
    st.count[j] = cnt;
    st.nobs[j] = nobs;
    st.n3[j] = c3;
    st.mean[j] = mu;
    st.inv_sd[j] = s;
}

// K-split geometry of a matrix-core product: nsplit splits of st_per super-tiles,
// nrb row blocks, xcd = 1 when the workgroups of one split share an XCD.
struct BfSplit {
    int nsplit = 1;
    int64_t st_per = 1;
    int nrb = 1;
    int xcd = 0;
};
struct MixedShape {
    int64_t n = 0, p = 0;
    int64_t nI = 0, ldI = 0;      // layout I: rows (individuals, padded) and bytes per row
    int64_t pS = 0, ldS = 0;      // layout S: rows (SNPs, padded) and bytes per row
    int64_t nstW = 0, nstX = 0;   // 256-wide super-tiles along SNPs / individuals
    int64_t stW = 0, stX = 0;     // super-tiles per K split
    int splitW = 1, splitX = 1;
    bool int8 = false;            // operand format: int8 limbs (true) or split BF16
    bool exact = false;           // FP64-exact block products: seven int8 limbs, two
                                  // vectors per pass (overrides int8)
    BfSplit bfW[3], bfX[3];       // split BF16 by column class: b <= 8, <= 16, <= 32
    BfSplit limbW, limbX;         // single-vector FP64 products in seven int8 limbs
};
// Internal copies of the genotype matrix, built once at create.  Padding codes
// are 3 (missing), so padded individuals and SNPs contribute exactly zero
// without masking in the hot loops.
//   T: nT x Pq bytes; T[J * nT + i] = codes of SNPs 4J..4J+3 of individual i
//      (feeds A v: one byte = four SNPs of one individual)
//   P: nqP x pP bytes; P[I * pP + j] = codes of individuals 4I..4I+3 of SNP j
//      (feeds A^T u: one byte = four individuals of one SNP)
// With limb_mv (limb_rmv) set, A v (A^T u) runs on the int8 matrix cores
// instead and reads the tiled layout I (S) of the blocked path (geometry ms);
// T (P) is then not built.
struct Packed {
    const uint8_t* T = nullptr;
    const uint8_t* P = nullptr;
    int64_t n = 0, p = 0;
    int64_t nT = 0, Pq = 0;       // rows (padded individuals), SNP quads of T
    int64_t pP = 0, nq = 0, nqP = 0;  // padded SNPs, individual quads (real, padded) of P
    bool limb_mv = false, limb_rmv = false;
    const uint8_t* I = nullptr;
    const uint8_t* S = nullptr;
    MixedShape ms;
};

// Device scratch used by the two-stage reductions of the matvec kernels.
struct MatvecWork {
    double* partial = nullptr;        // split partials
    size_t partial_elems = 0;
    void* lfrag = nullptr;            // limb products: B operand fragments of the vector
    double* lcpart = nullptr;         // limb products: 64 chunk sums of the vector
    double* lcmax = nullptr;          // limb products: 64 chunk maxima
    unsigned int* counters = nullptr; // zeroed, one per output block
    size_t ncounters = 0;
    double* npart = nullptr;          // per-block sums of squares for a NormTail
};

struct NormTail;

// ---- k_stats.hip ----
void launch_colstats(const uint8_t* G, int64_t n, int64_t p, int64_t ld, const ColStats& st,
                     hipStream_t s);
void launch_unpack(const uint8_t* G, int64_t n, int64_t p, int64_t ld, int8_t* out,
                   hipStream_t s);
// Plain streaming read of `bytes` bytes (the read-rate diagnostic).
void launch_read_rate(const void* buf, int64_t bytes, hipStream_t s);
// Layout shapes, sizes and the builders (from the caller's SNP-major G).
void layout_shape(int64_t n, int64_t p, Packed& L);
size_t layout_T_bytes(const Packed& L);
size_t layout_P_bytes(const Packed& L);
void build_layouts(const uint8_t* G, int64_t ld, const Packed& L, hipStream_t s);


// ---- k_matvec.hip: FP64 products with the implicit standardised matrix ----
// y = A v - (beta ? *beta : 0) * uprev      (y, uprev: n; v: p)
// With a tail, ||y|| also goes to tail->nrm_out (and the PRO update runs);
// the tail's npart is taken from w.  With ev, ev[0] and ev[1] are recorded
// right before and after the product kernel (not its reduce).
void launch_matvec(const Packed& P, const ColStats& st, const double* v, double* y,
                   const double* beta, const double* uprev, MatvecWork& w, hipStream_t s,
                   const NormTail* tail = nullptr, const hipEvent_t* ev = nullptr);
// z = A^T u - (alpha ? *alpha : 0) * vprev  (u: n; z, vprev: p)
void launch_rmatvec(const Packed& P, const ColStats& st, const double* u, double* z,
                    const double* alpha, const double* vprev, MatvecWork& w, hipStream_t s,
                    const NormTail* tail = nullptr, const hipEvent_t* ev = nullptr);
// Length of MatvecWork::npart.
size_t matvec_norm_partials(const Packed& P);
size_t matvec_partial_elems(const Packed& P);
size_t matvec_counters(const Packed& P);

// ---- batched solver: many problems stepped together ----
constexpr int kMaxBatch = 1024;
// Per-problem view read by the batched kernels (device array, one per problem).
// Every Lanczos quantity has the same meaning as in the single-problem solver;
// state[0] = current step j and state[1] = nlock (Ritz vectors kept at the last
// restart), shared by all problems because they step in lockstep.
struct BatchDesc {
    const uint8_t* T;
    const uint8_t* P;
    int64_t n, p, nT, Pq, pP, nq;
    const double* mean;
    const double* inv_sd;
    int64_t mv_per_split, rmv_per_split;
    int32_t mv_nsplit, rmv_nsplit, mv_rowblocks, rmv_colblocks;
    double* partial;                 // product split partials
    double* U;                       // n x maxm
    double* V;                       // p x (maxm + 1)
    double* alpha;
    double* beta;
    double* theta;
    double* rho;
    double* tnpart;                  // projection partials (batch_tn_partial_elems)
    double* h;                       // projection coefficients, hstride
    double* npart;                   // norm partials, chunks
    double* anorm;                   // running max of the alphas and betas
    int32_t* active;                 // 0 once converged or stopped
    int32_t* breakdown;              // 1 + half-step (2j + side) of a breakdown, else 0
    // A^T u in int8 limbs (when S is set): layout S (pP then holds its padded
    // rows and rmv_nsplit its K splits, as the reduce kernel reads them), the
    // limb fragments of u_j and its column sum / maximum chunks
    const uint8_t* S;
    int64_t ldS, nstX, limb_st_per;
    int32_t limb_nrb;
    void* lfrag;
    double* lcpart;
    double* lcmax;
};

// Product geometry of one problem for the given split targets (blocks per launch).
struct ProductPlan {
    int64_t mv_per_split = 0, rmv_per_split = 0;
    int mv_nsplit = 1, rmv_nsplit = 1, mv_rowblocks = 1, rmv_colblocks = 1;
};
ProductPlan product_plan(const Packed& L, int64_t mv_target, int64_t rmv_target);
size_t product_plan_partial_elems(const Packed& L, const ProductPlan& pl);
// Persistent products over the tiles of every active problem: tile0[q] is the
// first tile of problem q (tile0[count] = total), `grid` workgroups stride over
// the tiles.  Left: partial of A v_j.  Right: partial of A^T u_j.
void launch_bmatvec(const BatchDesc* d, const int* tile0, int count, const int* state, int grid,
                    hipStream_t s);
void launch_brmatvec(const BatchDesc* d, const int* tile0, int count, const int* state, int grid,
                     hipStream_t s);
// K splits of one problem's A^T u in limbs inside a batch: about `target` tiles
// (split x row block) per problem, at least one split, at most 2^20 per split.
BfSplit limb_batch_split(const MixedShape& m, int64_t target);
// Persistent A^T u_j in int8 limbs for the problems whose descriptor has S set
// (all of the batch): column sums, limb fragments, then the matrix-core kernel
// over the (split, row block) tiles of every active problem.
void launch_blimb_rmatvec(const BatchDesc* d, const int* tile0, int count, const int* state,
                          int grid, int64_t max_nst, hipStream_t s);
// u_j = sum of partials - beta_{j-1} u_{j-1} (or - U(:, 0:nlock) rho right after a
// restart); v_{j+1} = s o (sum of partials) - alpha_j v_j.
void launch_bmatvec_reduce(const BatchDesc* d, const int* state, int count, int64_t max_n,
                           hipStream_t s);
void launch_brmatvec_reduce(const BatchDesc* d, const int* state, int count, int64_t max_p,
                            hipStream_t s);
// ---- k_batch.hip ----
// Full CGS2 of the new vector of every active problem (side 0: u_j against
// U(:, 0:j); side 1: v_{j+1} against V(:, 0:j+1)), then its norm into alpha_j /
// beta_j and the scaling.  hstride >= maxm + 2.
void launch_bortho(const BatchDesc* d, const int* state, int count, int side, int64_t max_len,
                   int hstride, hipStream_t s);
size_t bortho_chunks(int64_t len);
// h = Q^T r of every active problem on the FP64 matrix cores (k_block.hip).
size_t batch_tn_partial_elems(int hstride);
void launch_batch_proj(const BatchDesc* d, const int* state, int count, int side, int hstride,
                       hipStream_t s);
void launch_bstep(int* state, hipStream_t s);
// v_0 of every problem scaled to unit norm (start of a solve).
void launch_bstart(const BatchDesc* d, int count, int64_t max_p, int hstride, hipStream_t s);
// Leave-one-block-out batches: problem q's right vectors are zero on its own
// SNP block [lohi[2q], lohi[2q+1]) (device array); all problems share one matrix.
// out(:, q) = v_j (side 0, len p) or u_j (side 1, len n); zero when inactive.
void launch_loco_gather(const BatchDesc* d, const int* state, int count, int side, double* out,
                        int64_t len, hipStream_t s);
// u_j = Y(:, q) - beta_{j-1} u_{j-1} (or - U(:, 0:nlock) rho after a restart).
void launch_loco_left(const BatchDesc* d, const int* state, int count, const double* Y, int64_t n,
                      hipStream_t s);
// v_{j+1} = Z(:, q) without the rows of block q, - alpha_j v_j.
void launch_loco_right(const BatchDesc* d, const int* state, int count, const double* Z, int64_t p,
                       const int64_t* lohi, hipStream_t s);
// v_0 of every problem zeroed on its own block.
void launch_loco_mask(const BatchDesc* d, int count, const int64_t* lohi, hipStream_t s);

// ---- k_ortho.hip: Gram-Schmidt, norms, small dense ops on the Krylov bases ----
struct OrthoWork {
    double* partial = nullptr;      // nblocks x (maxcols + 1)
    size_t partial_elems = 0;
    unsigned int* counters = nullptr;
    double* h = nullptr;            // projection coefficients (maxcols + 1)
    double* tn_partial = nullptr;   // Q^T r partials (gemm_tn_partial_elems)
    double* npart = nullptr;        // ||r||^2 partials of the last CGS2 pass (cgs_norm_partials)
    double* cgs_partial = nullptr;  // CGS2 projection partials, both passes
    size_t cgs_partial_elems = 0;
};
size_t ortho_partial_elems(int64_t len, int maxcols);
size_t cgs_partial_elems(int64_t len, int maxcols);
int cgs_norm_partials(int64_t len);

// r <- r - Q (Q^T r) with Q = [Q(:, 0:ncols)], column-major leading dim ldq.
// `enable` (device, may be NULL = always) gates the whole call: 0 skips it.
// If adaptive, the second pass runs only when ||r1|| < ||r0|| / sqrt(2);
// otherwise two passes always.  Counts performed passes into *passes (device).
// Block CGS2 of Y (len x b, 1 <= b <= 4, ld ldy) against Q (len x ncols): the
// single-vector kernels' three fused passes for all b vectors at once.
size_t block_cgs2_partial_elems(int64_t len, int maxcols, int b);
void launch_block_cgs2(const double* Q, int64_t ldq, int64_t len, int ncols, double* Y, int64_t ldy,
                       int b, double* partial, size_t partial_elems, hipStream_t s);
void launch_cgs2(const double* Q, int64_t ldq, int64_t len, int ncols, double* r,
                 const int* enable, int adaptive, int* passes, OrthoWork& w, hipStream_t s);
// nrm = ||r||; if nrm <= thresh(*) then breakdown: *flag = 1 and nrm stored as 0,
// r left unscaled; else out = r / nrm (out may alias r).
//   thresh = eps * max(*norm_est, nrm) * sqrt(max_dim); *norm_est updated.
// On breakdown, *first_breakdown (if not NULL and still < 0) receives `step`.
// Scale r to unit length right after a non-adaptive launch_cgs2 on the same r
// (uses the norm partials that CGS2 left in w.npart); with *enable == 0 (CGS2
// skipped) *nrm_out must already hold ||r||.  Same breakdown test and outputs as
// launch_normalize.
void launch_normalize_after_cgs2(double* r, int64_t len, double* nrm_out, double* norm_est,
                                 double root_maxdim, int* flag, const int* enable, OrthoWork& w,
                                 hipStream_t s, int* first_breakdown, int step);
void launch_normalize(double* r, int64_t len, double* out, double* nrm_out, double* norm_est,
                      double root_maxdim, int* flag, OrthoWork& w, hipStream_t s,
                      int* first_breakdown = nullptr, int step = 0);
// One-sided reorthogonalisation: *flag = 1 when the largest |Q(:, 0:ncols)^T q|
// exceeds omega * *qnorm (device scalar, ||q||); the flag is only ever set, never
// cleared.
void launch_overlap_check(const double* Q, int64_t len, int ncols, const double* q, double omega,
                          const double* qnorm, int* flag, OrthoWork& w, hipStream_t s);
// y -= Q(:, 0:ncols) * c  (c device, ncols)
void launch_gemv_n_sub(const double* Q, int64_t ldq, int64_t len, int ncols, const double* c,
                       double* y, hipStream_t s);
// C(len x ncols_out) = Q(len x ncols_in) * S(ncols_in x ncols_out) (S column-major, lds)
void launch_gemm_tall(const double* Q, int64_t ldq, int64_t len, int ncols_in, const double* S,
                      int lds, int ncols_out, double* C, int64_t ldc, hipStream_t s);
// Gaussian vector from a counter-based generator (Box-Muller), seed-keyed.
void launch_gaussian(double* x, int64_t len, uint64_t seed, uint64_t stream_id, hipStream_t s);
// Sign rule: for each of k columns of V (ldv), find the largest |entry| (lowest
// index on ties); if negative flip that V column and the U column.
void launch_sign_fix(double* U, int64_t ldu, int64_t n, double* V, int64_t ldv, int64_t p,
                     int k, hipStream_t s);

// ---- k_svd.hip: Ritz extraction ----
// One-sided Jacobi SVD of a dense m x m matrix in one workgroup:
// B = P diag(S) Q^T, S descending.  Up to kMaxKrylov the matrix and the
// accumulated rotations live in LDS.  Beyond that, with `rlog` (device, at
// least svd_log_elems(m) doubles) and svd_logged_fits_lds(m), only the matrix
// lives in LDS: the rotations are logged and replayed onto Q afterwards (same
// result bit for bit).  Otherwise the working matrices live in `gscratch`
// (device, at least svd_scratch_elems(m) doubles).  qcols (0 = all): leading
// columns of Q the caller reads; on the logged path, when the last of them has
// a singular value of at least 5% of the largest, they are formed as
// B^T P diag(1/S) (error below about 1e-13) instead of by the replay, and the
// columns from qcols on are left unwritten.
void launch_dense_svd(const double* B, int m, double* P, double* S, double* Q, double* gscratch,
                      hipStream_t s, double* rlog = nullptr, int qcols = 0);
size_t svd_log_elems(int m);
bool svd_logged_fits_lds(int m);
size_t svd_scratch_elems(int m);
// True when the m x m SVD working set fits the device's LDS per workgroup.
bool svd_fits_lds(int m);
constexpr int kMaxSvd = 1024;

// Builds the projected matrix from the device state and runs the SVD, then the
// convergence test:
//   B(i,i) = alpha[i], B(i,i+1) = beta[i] for i >= nlock (bidiagonal part),
//   B(i,i) = theta[i], B(i,nlock) = rho[i] for i < nlock (restart arrowhead).
//   res_i = beta[m-1] * |P(m-1, i)|; conv = #leading i < k with res_i <= tol*S[0].
struct RitzOut {
    double* B;      // m x m scratch
    double* P;      // m x m
    double* S;      // m
    double* Q;      // m x m
    double* res;    // m
    int* nconv;     // 1
};
// head (optional): dense nlock x nlock block (ld nlock) in place of diag(theta),
// after a harmonic restart.
void launch_ritz(const double* alpha, const double* beta, const double* theta, const double* rho,
                 int nlock, int m, int k, double tol, const RitzOut& out, double* gscratch,
                 hipStream_t s, const double* head = nullptr);
// Harmonic thick restart: Bp ((m+1) x (m+1)) = [B, beta_last e_m; 0]; after its
// SVD (Ph, Qh), the plan: Z ((m+1) x (l+1), ld m+1) for V_new = V_{m+1} Z,
// head (l x l, ld l) and coupling c (l); U_new = U_m Ph(0:m, 0:l).
// work >= m * (l + 1) doubles.
void launch_harmonic_pad(const double* B, int m, const double* beta_last, double* Bp,
                         hipStream_t s);
void launch_harmonic_plan(const double* B, int m, const double* beta_last, const double* Ph,
                          const double* Qh, int l, double* work, double* Z, double* head,
                          double* c, hipStream_t s);
// The same for many problems at once (one workgroup each); problems with
// run == 0 are skipped.  gscratch: count * svd_scratch_elems(m) doubles when
// the matrix does not fit LDS.
struct BatchRitzArgs {
    const double* alpha;
    const double* beta;
    const double* theta;
    const double* rho;
    RitzOut out;
    int32_t run;
};
void launch_ritz_batched(const BatchRitzArgs* args, int count, int nlock, int m, int k, double tol,
                         double* gscratch, hipStream_t s);

// ---- k_pro.hip: partial reorthogonalisation estimates ----
struct ProState {
    double* mu;     // left estimates  u_j^T u_i, length maxm
    double* nu;     // right estimates v_{j+1}^T v_i, length maxm + 1
    int* flag_left;   // 1 = reorthogonalise the next left vector
    int* flag_right;  // 1 = reorthogonalise the next right vector
    int* force;       // [0] left, [1] right: pending forced passes (Simon's rule)
};
// Everything one PRO update reads besides the new norm: the update follows
// alpha_j (left side) or beta_j (right side); theta/rho/nlock describe the
// thick-restart block (nlock = 0 without restart); noise_scale = eps *
// sqrt(max(n, p)), and the noise added per update is noise_scale * (*norm_est)
// / alpha_j (or beta_j).
struct ProArgs {
    const double* alpha;
    const double* beta;
    const double* theta;
    const double* rho;
    int nlock;
    int j;
    double omega;
    double noise_scale;
    const double* norm_est;
    ProState st;
};
// PRO update after alpha_j (left) or beta_j (right) is in memory.
void launch_pro_left(const ProArgs& a, hipStream_t s);
void launch_pro_right(const ProArgs& a, hipStream_t s);
// Norm (and PRO update) of a product's output, requested from launch_matvec /
// launch_rmatvec: their reduce kernel leaves per-workgroup sums of squares in
// npart and one more small kernel finishes (pro.h).  pro = 0 norm only, 1 left
// update, 2 right update.
struct NormTail {
    double* npart;
    double* nrm_out;
    int pro;
    ProArgs pa;
};
// Zero the estimates and force `force` full reorthogonalisations on each side.
void launch_pro_reset(const ProState& st, int maxm, int force, hipStream_t s);

// ---- k_svd.hip, restart helpers ----
// theta[i] = S[i], rho[i] = beta_last * P(m-1, i) for i < keep.
void launch_restart_scalars(const double* S, const double* P, int m, const double* beta_last,
                            int keep, double* theta, double* rho, hipStream_t s);

// ---- k_mixed.hip: MFMA block products (split BF16 or int8 limbs) ----
struct MixedWork {
    void* frag = nullptr;         // int8 limb fragments of the vector block
    double* partial = nullptr;
    double* cpart = nullptr;      // 32 x 64 column-sum partials
    double* cmax = nullptr;       // 32 x 64 column-maximum partials
};
MixedShape mixed_shape(int64_t n, int64_t p);
size_t mixed_frag_bytes(const MixedShape& m);
size_t mixed_partial_elems(const MixedShape& m);
// Either layout pointer may be NULL (that layout is not built).  With st, the
// pass that builds S also writes the column statistics (as launch_colstats).
void build_mixed_layouts(const uint8_t* G, int64_t n, int64_t p, int64_t ld, uint8_t* I,
                         uint8_t* S, hipStream_t s, const ColStats* st = nullptr);
// FP64 A v and A^T u in seven int8 limbs (layouts I and S): the colsum,
// fragment and matrix-core kernels, leaving per-split partials in w.partial
// (stride ms.nI for A v, ms.pS for A^T u) in the form the FP64 reduce kernels
// take.  Returns the number of K splits.
size_t limb_frag_bytes(const MixedShape& m);
size_t limb_partial_elems(const MixedShape& m);
int launch_matvec_limb(const MixedShape& m, const uint8_t* I, const ColStats& st, const double* v,
                       MatvecWork& w, hipStream_t s, const hipEvent_t* ev);
int launch_rmatvec_limb(const MixedShape& m, const uint8_t* S, const ColStats& st, const double* u,
                        MatvecWork& w, hipStream_t s, const hipEvent_t* ev);
// Y (n x b, ldy) = A W (W: p x b, ldw); Z (p x b, ldz) = A^T X (X: n x b, ldx); b <= 32.
// core_ev (optional): two events recorded around the matrix-core kernels
void launch_matmat_mixed(const MixedShape& m, const uint8_t* I, const ColStats& st,
                         const double* W, int64_t ldw, int b, double* Y, int64_t ldy,
                         MixedWork& w, hipStream_t s, const hipEvent_t* core_ev = nullptr);
void launch_rmatmat_mixed(const MixedShape& m, const uint8_t* S, const ColStats& st,
                          const double* X, int64_t ldx, int b, double* Z, int64_t ldz,
                          MixedWork& w, hipStream_t s, const hipEvent_t* core_ev = nullptr);

// ---- k_block.hip: FP64 block operations ----
size_t gemm_tn_partial_elems(int64_t len, int q);
// H (q x b, ldh) = Q^T Y
void launch_gemm_tn(const double* Q, int64_t ldq, const double* Y, int64_t ldy, int64_t len, int q,
                    int b, double* H, int ldh, double* partial, hipStream_t s);
// The same, skipped on the device when *enable == 0 or *skip != 0 (either may be NULL).
void launch_gemm_tn_gated(const double* Q, int64_t ldq, const double* Y, int64_t ldy, int64_t len,
                          int q, int b, double* H, int ldh, double* partial, const int* enable,
                          const int* skip, hipStream_t s);
// Out (len x nc) = Q H (subtract == 0) or Out -= Q H; Q (len x q), H (q x nc, ldh)
void launch_gemm_nn(const double* Q, int64_t ldq, int q, const double* H, int ldh, double* Out,
                    int64_t ldo, int64_t len, int nc, int subtract, hipStream_t s);
// Y -= Q H
void launch_gemm_nn_sub(const double* Q, int64_t ldq, double* Y, int64_t ldy, int64_t len, int q,
                        int b, const double* H, int ldh, hipStream_t s);
// shifted CholeskyQR3 of Y in place; R (b x b upper) to Rout; work >= 3 b^2.
// guard (2 doubles, optional): running column-norm scale and the flag for a
// column of R below 1e-4 of it, read by launch_block_finish.
void launch_block_qr(double* Y, int64_t ldy, int64_t len, int b, double* Rout, double* work,
                     double* partial, int* bad, hipStream_t s, double* guard = nullptr);
// Repairs a flagged block (Y, len x b, against the basis Qb, len x q, and
// within the block; R updated) and writes R (transpose: R^T) into Bm at (r0, c0).
void launch_block_finish(double* Y, int64_t ldy, int64_t len, int b, const double* Qb,
                         int64_t ldq, int q, double* R, const double* guard, double* Bm, int ldb,
                         int r0, int c0, int transpose, hipStream_t s);
void launch_put_block(double* Bm, int ldb, int r0, int c0, const double* X, int rows, int cols,
                      int ldx, int transpose, hipStream_t s);
void launch_copy_lead(const double* Bm, int ldb, int m, double* out, hipStream_t s);
void launch_block_residual(const double* C, int b, const double* P, int m, const double* S, int k,
                           double tol, double* res, int* nconv, hipStream_t s);
void launch_restart_block(double* Bm, int ldb, int keep, int b, const double* S, const double* C,
                          const double* P, int m, hipStream_t s);

}  // namespace gkl
