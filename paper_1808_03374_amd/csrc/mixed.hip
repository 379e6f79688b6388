// Blocked mixed-precision GKL (host engine).
//
// Block Lanczos bidiagonalisation of width b (the BLAS3 extension named in
// Section 5 of the paper), with thick restart from ordinary Ritz vectors
// (Section 3):
//     U_s R_s     = A V_s - U_{s-1} C_{s-1}^T      (block CGS2 against all U, QR)
//     V_{s+1} C_s = A^T U_s - V_s R_s^T            (block CGS2 against all V, QR)
// so that A [V_1..V_s] = [U_1..U_s] B with B block upper bidiagonal (R_s on the
// diagonal, C_s^T above it).  The two products run on the matrix cores, with
// split-BF16 vector tiles (GKL_PREC_MIXED), exact int8 limbs of a per-column
// fixed point (GKL_PREC_MIXED_INT8) or seven int8 limbs of 52-bit integers, FP64
// to the rounding of a sum (GKL_PREC_BLOCK_FP64); everything else (Gram-Schmidt, QR, B, its
// SVD, restart) is FP64.
// Ritz residual of triplet i: || C_s P(last block rows, i) ||.
// After a restart that keeps l Ritz vectors, B starts as diag(sigma_1..l) with the
// spike block G^T = (C_s P(last, 1:l))^T in columns l..l+b, and the next left
// block subtracts U~ G^T.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "engine.h"

namespace gkl {

struct MixedState {
    MixedShape shape;
    uint8_t* I = nullptr;
    uint8_t* S = nullptr;
    MixedWork w;
    int b = 16;
    int mmax = 0;       // left basis capacity (columns)
    int keep = 0;
    int ldb = 0;        // leading dimension of the projected matrix
    double* U = nullptr;
    double* V = nullptr;
    double* H = nullptr;       // (mmax + b) x b projection coefficients
    double* Bm = nullptr;      // ldb x ldb projected matrix
    double* Bc = nullptr;      // compact copy for the SVD
    double* R = nullptr;       // b x b
    double* RT = nullptr;      // b x b
    double* C = nullptr;       // b x b last right factor
    double* qrwork = nullptr;  // 3 b^2
    double* tmp = nullptr;     // max(n, p) x keep
    double* gpart = nullptr;
    size_t gpart_elems = 0;
    double* svd_scratch = nullptr;
    double* svd_log = nullptr;         // rotation log of the SVD for 96 < m <= 128
    int* iflags = nullptr;     // [0] nconv [1] bad pivots
    double* guard = nullptr;   // [0] column-norm scale [1] block QR flag
    RitzOut ritz{};
};

bool mixed_supported() { return true; }
void destroy_mixed(MixedState* m) { delete m; }

}  // namespace gkl

using namespace gkl;

void gkl_ctx::setup_mixed()
{
    mixed = new MixedState();
    MixedState& M = *mixed;
    DeviceArena& A = prob.arena;
    hipStream_t s = prob.stream;
    const int64_t n = prob.n, p = prob.p;
    // Defaults (measured on 10,000 x 100,000 and 50,000 x 500,000 genotypes,
    // k = 20): block width 8, a basis of 128 columns (the largest projected
    // matrix whose SVD runs in LDS, with its rotations logged and replayed; 1.4x
    // faster than 96 columns at the larger size, the same at the smaller) and a
    // quarter of the free columns kept at a restart.
    M.b = opt.block_width > 0 ? opt.block_width : 8;
    if (M.b > 32) fail(GKL_ERR_INVALID, "block_width must be <= 32");
    const int64_t mn = std::min(n, p);
    int m = opt.krylov_dim > 0 ? opt.krylov_dim : std::max(kMaxBlockedKrylov, 3 * k + M.b);
    m = ((m + M.b - 1) / M.b) * M.b;
    if (m > mn) m = (int)(mn / M.b) * M.b;
    if (m < 2 * M.b || m <= k) fail(GKL_ERR_INVALID, "problem too small for the blocked solver");
    M.mmax = m;
    M.keep = opt.keep > 0 ? opt.keep : k + (m - k) / 4;
    M.keep = std::min(M.keep, m - M.b);
    if (M.keep < k) M.keep = k;
    M.ldb = m + M.b;
    M.shape = mixed_shape(n, p);
    M.shape.int8 = opt.precision == GKL_PREC_MIXED_INT8;
    M.shape.exact = opt.precision == GKL_PREC_BLOCK_FP64;
    M.I = static_cast<uint8_t*>(A.alloc((size_t)M.shape.nI * M.shape.ldI));
    M.S = static_cast<uint8_t*>(A.alloc((size_t)M.shape.pS * M.shape.ldS));
    build_mixed_layouts(prob.G_user, n, p, prob.ld, M.I, M.S, s);
    M.w.frag = A.alloc(mixed_frag_bytes(M.shape));
    M.w.partial = static_cast<double*>(A.alloc(sizeof(double) * mixed_partial_elems(M.shape)));
    M.w.cpart = static_cast<double*>(A.alloc(sizeof(double) * 32 * 64));
    M.w.cmax = static_cast<double*>(A.alloc(sizeof(double) * 32 * 64));
    const int b = M.b;
    M.U = static_cast<double*>(A.alloc(sizeof(double) * (size_t)n * m));
    M.V = static_cast<double*>(A.alloc(sizeof(double) * (size_t)p * (m + b)));
    M.H = static_cast<double*>(A.alloc(sizeof(double) * (size_t)(m + b) * b));
    M.Bm = static_cast<double*>(A.alloc(sizeof(double) * (size_t)M.ldb * M.ldb));
    M.Bc = static_cast<double*>(A.alloc(sizeof(double) * (size_t)m * m));
    M.R = static_cast<double*>(A.alloc(sizeof(double) * b * b));
    M.RT = static_cast<double*>(A.alloc(sizeof(double) * b * b));
    M.C = static_cast<double*>(A.alloc(sizeof(double) * b * b));
    M.qrwork = static_cast<double*>(A.alloc(sizeof(double) * 3 * b * b));
    M.tmp = static_cast<double*>(A.alloc(sizeof(double) * (size_t)std::max(n, p) * M.keep));
    const size_t gp = std::max(gemm_tn_partial_elems(std::max(n, p), m + b),
                               gemm_tn_partial_elems(std::max(n, p), b));
    M.gpart_elems = std::max(gp, block_cgs2_partial_elems(std::max(n, p), m + b, b));
    M.gpart = static_cast<double*>(A.alloc(sizeof(double) * M.gpart_elems));
    M.iflags = static_cast<int*>(A.alloc(sizeof(int) * 8));
    M.guard = static_cast<double*>(A.alloc(sizeof(double) * 2));
    M.ritz.B = M.Bc;
    M.ritz.P = static_cast<double*>(A.alloc(sizeof(double) * (size_t)m * m));
    M.ritz.Q = static_cast<double*>(A.alloc(sizeof(double) * (size_t)m * m));
    M.ritz.S = static_cast<double*>(A.alloc(sizeof(double) * m));
    M.ritz.res = static_cast<double*>(A.alloc(sizeof(double) * m));
    M.ritz.nconv = M.iflags;
    if (!svd_fits_lds(m)) {
        if (svd_logged_fits_lds(m))
            M.svd_log = static_cast<double*>(A.alloc(sizeof(double) * svd_log_elems(m)));
        else
            M.svd_scratch = static_cast<double*>(A.alloc(sizeof(double) * svd_scratch_elems(m)));
    }
    GKL_HIP(hipMemsetAsync(M.iflags, 0, sizeof(int) * 8, s));
    maxm = m;
    keep = M.keep;
    krylov = m;
}

// Block CGS2 of the b columns of Y (len) against Q(:, 0:q).
static void block_cgs2(MixedState& M, const double* Q, int64_t len, int q, double* Y, hipStream_t s)
{
    if (q <= 0) return;
    const int b = M.b;
    if (b <= 4) {
        // the fused three-pass kernels: one read of Q per pass for the whole block
        launch_block_cgs2(Q, len, len, q, Y, len, b, M.gpart, M.gpart_elems, s);
        return;
    }
    for (int pass = 0; pass < 2; ++pass) {
        launch_gemm_tn(Q, len, Y, len, len, q, b, M.H, M.mmax + b, M.gpart, s);
        launch_gemm_nn_sub(Q, len, Y, len, len, q, b, M.H, M.mmax + b, s);
    }
}

gkl_status gkl_ctx::solve_mixed(double* sigma, double* Uo, int64_t ldu, double* Vo, int64_t ldv)
{
    MixedState& M = *mixed;
    hipStream_t s = prob.stream;
    const int64_t n = prob.n, p = prob.p;
    const int b = M.b;
    // start block
    if (opt.v0) GKL_HIP(hipMemcpyAsync(M.V, opt.v0, sizeof(double) * p * b, hipMemcpyDeviceToDevice, s));
    else launch_gaussian(M.V, p * b, opt.seed, 0, s);
    GKL_HIP(hipMemsetAsync(M.Bm, 0, sizeof(double) * (size_t)M.ldb * M.ldb, s));
    GKL_HIP(hipMemsetAsync(M.iflags, 0, sizeof(int) * 8, s));
    GKL_HIP(hipMemsetAsync(M.guard, 0, sizeof(double) * 2, s));
    launch_block_qr(M.V, p, p, b, M.R, M.qrwork, M.gpart, M.iflags + 1, s);
    int o = 0;
    int nlock_m = 0;         // columns kept at the last restart (0 = none)
    int mcur = 0;
    int nconv = 0;
    int svd_m = -1;
    bool converged = false;
    int since_check = 0;
    // convergence is tested when the basis is full unless asked more often; with
    // the default basis and schedule, from 4e9 genotypes (1 GB packed) on, also
    // before the first restart, from k + b columns on each time the basis has
    // grown by a quarter -- a well separated spectrum then stops long before a
    // 128-column basis is full.  Below that size a block step (two passes over
    // at most 1 GB plus its small launches) costs less than a test (a projected
    // SVD of up to 128 columns and a host synchronisation), so the early tests
    // would mostly add time (10,000 x 100,000: about 6 tests, +6% per solve).
    const int check_every = opt.check_every > 0 ? opt.check_every : 1 << 30;
    const bool grow_checks = opt.check_every <= 0 && opt.krylov_dim <= 0 && (double)n * p >= 4e9;
    int last_check_m = 0;
    while (true) {
        double* Ub = M.U + (int64_t)o * n;
        double* Vb = M.V + (int64_t)o * p;
        double* Vn = M.V + (int64_t)(o + b) * p;
        // left block: A V_o minus the coupling to the previous left block
        const int ev = timing_begin(false);
        launch_matmat_mixed(M.shape, M.I, prob.st, Vb, p, b, Ub, n, M.w, s,
                            ev >= 0 ? &ev_pool[ev + 2] : nullptr);
        timing_end(ev, false, true);
        info.matvecs += b;
        info.passes_over_G += M.shape.exact ? (b + 1) / 2 : M.shape.int8 ? (b + 15) / 16 : 1;
        if (o > 0) {
            if (o == nlock_m)
                launch_gemm_nn_sub(M.U, n, Ub, n, n, nlock_m, b, M.Bm + (int64_t)o * M.ldb, M.ldb, s);
            else
                launch_gemm_nn_sub(M.U + (int64_t)(o - b) * n, n, Ub, n, n, b, b,
                                   M.Bm + (int64_t)o * M.ldb + (o - b), M.ldb, s);
            block_cgs2(M, M.U, n, o, Ub, s);
            info.reorths += 2;
        }
        // a block that ran out of new directions (low rank) is repaired before
        // its R enters the projected matrix
        launch_block_qr(Ub, n, n, b, M.R, M.qrwork, M.gpart, M.iflags + 1, s, M.guard);
        launch_block_finish(Ub, n, n, b, M.U, n, o, M.R, M.guard, M.Bm, M.ldb, o, o, 0, s);
        // right block: A^T U_o - V_o R^T
        const int ev2 = timing_begin(true);
        launch_rmatmat_mixed(M.shape, M.S, prob.st, Ub, n, b, Vn, p, M.w, s,
                             ev2 >= 0 ? &ev_pool[ev2 + 2] : nullptr);
        timing_end(ev2, true, true);
        info.matvecs += b;
        info.passes_over_G += M.shape.exact ? (b + 1) / 2 : M.shape.int8 ? (b + 15) / 16 : 1;
        launch_put_block(M.RT, b, 0, 0, M.R, b, b, b, 1, s);
        launch_gemm_nn_sub(Vb, p, Vn, p, p, b, b, M.RT, b, s);
        block_cgs2(M, M.V, p, o + b, Vn, s);
        info.reorths += 2;
        launch_block_qr(Vn, p, p, b, M.C, M.qrwork, M.gpart, M.iflags + 1, s, M.guard);
        launch_block_finish(Vn, p, p, b, M.V, p, o + b, M.C, M.guard, M.Bm, M.ldb, o, o + b, 1, s);
        o += b;
        mcur = o;
        info.steps += 1;
        ++since_check;
        const bool full = o + b > M.mmax;
        const bool budget = opt.max_matvecs > 0 && info.matvecs >= opt.max_matvecs;
        const bool grown = grow_checks && info.restarts == 0 && mcur >= k + b &&
                           4 * mcur >= 5 * last_check_m;
        if (mcur >= k && (full || budget || since_check >= check_every || grown)) {
            since_check = 0;
            last_check_m = mcur;
            launch_copy_lead(M.Bm, M.ldb, mcur, M.Bc, s);
            launch_dense_svd(M.Bc, mcur, M.ritz.P, M.ritz.S, M.ritz.Q, M.svd_scratch, s, M.svd_log,
                             M.keep);
            launch_block_residual(M.C, b, M.ritz.P, mcur, M.ritz.S, k, tol, M.ritz.res,
                                  M.ritz.nconv, s);
            svd_m = mcur;
            GKL_HIP(hipMemcpyAsync(&nconv, M.ritz.nconv, sizeof(int), hipMemcpyDeviceToHost, s));
            GKL_HIP(hipStreamSynchronize(s));
            info.nconv = nconv;
            if (nconv >= k) { converged = true; break; }
            if (budget) break;
            if (full) {
                // thick restart keeping M.keep Ritz vectors
                const int kp = M.keep;
                launch_gemm_nn(M.V, p, mcur, M.ritz.Q, mcur, M.tmp, p, p, kp, 0, s);
                GKL_HIP(hipMemcpyAsync(M.V, M.tmp, sizeof(double) * (size_t)p * kp,
                                       hipMemcpyDeviceToDevice, s));
                GKL_HIP(hipMemcpyAsync(M.V + (int64_t)kp * p, M.V + (int64_t)mcur * p,
                                       sizeof(double) * (size_t)p * b, hipMemcpyDeviceToDevice, s));
                launch_gemm_nn(M.U, n, mcur, M.ritz.P, mcur, M.tmp, n, n, kp, 0, s);
                GKL_HIP(hipMemcpyAsync(M.U, M.tmp, sizeof(double) * (size_t)n * kp,
                                       hipMemcpyDeviceToDevice, s));
                launch_restart_block(M.Bm, M.ldb, kp, b, M.ritz.S, M.C, M.ritz.P, mcur, s);
                nlock_m = kp;
                o = kp;
                svd_m = -1;
                info.restarts += 1;
            }
        } else if (budget) {
            break;
        }
    }
    if (svd_m != mcur) {
        launch_copy_lead(M.Bm, M.ldb, mcur, M.Bc, s);
        launch_dense_svd(M.Bc, mcur, M.ritz.P, M.ritz.S, M.ritz.Q, M.svd_scratch, s, M.svd_log,
                             M.keep);
        launch_block_residual(M.C, b, M.ritz.P, mcur, M.ritz.S, k, tol, M.ritz.res, M.ritz.nconv, s);
    }
    const int kk = std::min(k, mcur);
    GKL_HIP(hipMemcpyAsync(sigma, M.ritz.S, sizeof(double) * kk, hipMemcpyDeviceToDevice, s));
    launch_gemm_nn(M.U, n, mcur, M.ritz.P, mcur, Uo, ldu, n, kk, 0, s);
    launch_gemm_nn(M.V, p, mcur, M.ritz.Q, mcur, Vo, ldv, p, kk, 0, s);
    launch_sign_fix(Uo, ldu, n, Vo, ldv, p, kk, s);
    std::vector<double> res(kk), s0(1);
    int bad = 0;
    GKL_HIP(hipMemcpyAsync(res.data(), M.ritz.res, sizeof(double) * kk, hipMemcpyDeviceToHost, s));
    GKL_HIP(hipMemcpyAsync(s0.data(), M.ritz.S, sizeof(double), hipMemcpyDeviceToHost, s));
    GKL_HIP(hipMemcpyAsync(&bad, M.iflags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    GKL_HIP(hipStreamSynchronize(s));
    double sum = 0.0, mx = 0.0;
    for (int i = 0; i < kk; ++i) {
        sum += res[i];
        mx = std::max(mx, s0[0] > 0 ? res[i] / s0[0] : 0.0);
    }
    info.sum_residual_est = sum;
    info.max_residual_rel = mx;
    info.converged = converged ? 1 : 0;
    info.nconv = converged ? k : nconv;
    if (bad > 0 && !converged)
        last_error = "block orthonormalisation met a rank-deficient block";
    return converged ? GKL_OK : GKL_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// Batched solves -- built in batched.hip
// ---------------------------------------------------------------------------
extern "C" {

gkl_status gkl_matmat_mixed(gkl_ctx* ctx, const double* W, int32_t b, double* Y)
{
    if (!ctx || !W || !Y || b < 1 || b > 32) return GKL_ERR_INVALID;
    if (!ctx->mixed) {
        ctx->last_error = "context was not created with a blocked precision (GKL_PREC_MIXED, _MIXED_INT8 or _BLOCK_FP64)";
        return GKL_ERR_INVALID;
    }
    try {
        hipStream_t s = ctx->prob.stream;
        launch_matmat_mixed(ctx->mixed->shape, ctx->mixed->I, ctx->prob.st, W, ctx->prob.p, b, Y,
                            ctx->prob.n, ctx->mixed->w, s);
        GKL_HIP(hipStreamSynchronize(s));
        return GKL_OK;
    } catch (const Error& e) {
        ctx->last_error = e.msg;
        return e.status;
    }
}

gkl_status gkl_rmatmat_mixed(gkl_ctx* ctx, const double* X, int32_t b, double* Z)
{
    if (!ctx || !X || !Z || b < 1 || b > 32) return GKL_ERR_INVALID;
    if (!ctx->mixed) {
        ctx->last_error = "context was not created with a blocked precision (GKL_PREC_MIXED, _MIXED_INT8 or _BLOCK_FP64)";
        return GKL_ERR_INVALID;
    }
    try {
        hipStream_t s = ctx->prob.stream;
        launch_rmatmat_mixed(ctx->mixed->shape, ctx->mixed->S, ctx->prob.st, X, ctx->prob.n, b, Z,
                             ctx->prob.p, ctx->mixed->w, s);
        GKL_HIP(hipStreamSynchronize(s));
        return GKL_OK;
    } catch (const Error& e) {
        ctx->last_error = e.msg;
        return e.status;
    }
}

}  // extern "C"
