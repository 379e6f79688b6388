// FP64 block operations for block GKL bidiagonalisation (gfx950).
//
// Block Lanczos (named as future work in Section 5 of the paper) keeps the
// recurrence scalars, the Gram-Schmidt reorthogonalisation and the projected
// matrix in FP64; only the two products with the genotype matrix use the
// split-BF16 MFMA path.  This file holds the FP64 pieces:
//   * H = Q^T Y for tall Q (len x q) and Y (len x b): LDS-tiled, partials per row
//     block, summed by the last block in a fixed order;
//   * Y -= Q H;
//   * block orthonormalisation by shifted Cholesky QR applied three times
//     (shifted CholeskyQR3, Fukaya, Kannan, Nakatsukasa, Yamamoto & Yanagisawa,
//     SIAM J. Sci. Comput. 2020): Gram matrix, Cholesky in one workgroup,
//     triangular solve applied to every row, R accumulated;
//   * Ritz residuals of the block-bidiagonal projected matrix.
#include <math.h>

#include "kernels.h"

namespace gkl {

namespace {
constexpr int kTR = 32;       // rows per LDS tile
constexpr int kQC = 96;       // Q columns per block (grid.y covers more)
constexpr int kBmax = 32;     // block width limit
}  // namespace

// H(q x b, ldh) = Q(len x q)^T Y(len x b); grid (row chunks, q chunks of 96).
// Thread t computes outputs (qcol = t / 16 * 6 + 0..5 within the chunk, ycol =
// t % 16 and t % 16 + 16 when b > 16) over the chunk's rows.
__global__ void __launch_bounds__(256)
gemm_tn_kernel(const double* __restrict__ Q, int64_t ldq, const double* __restrict__ Y,
               int64_t ldy, int64_t len, int q, int b, int64_t rows_per_block,
               double* __restrict__ H, int ldh, double* __restrict__ partial,
               unsigned int* __restrict__ counters)
{
    __shared__ double qs[kTR][kQC + 1];
    __shared__ double ys[kTR][kBmax + 1];
    const int q0 = blockIdx.y * kQC;
    const int qn = q - q0 < kQC ? q - q0 : kQC;
    const int tq = (threadIdx.x >> 4) * 6;          // 16 groups x 6 = 96 columns
    const int ty = threadIdx.x & 15;
    double acc[2][6];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 6; ++v) acc[u][v] = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = r0 + rows_per_block < len ? r0 + rows_per_block : len;
    for (int64_t rt = r0; rt < r1; rt += kTR) {
        const int nr = (int)(r1 - rt < kTR ? r1 - rt : kTR);
        for (int e = threadIdx.x; e < kTR * kQC; e += 256) {
            const int rr = e % kTR, c = e / kTR;
            qs[rr][c] = (rr < nr && c < qn) ? Q[(int64_t)(q0 + c) * ldq + rt + rr] : 0.0;
        }
        for (int e = threadIdx.x; e < kTR * kBmax; e += 256) {
            const int rr = e % kTR, c = e / kTR;
            ys[rr][c] = (rr < nr && c < b) ? Y[(int64_t)c * ldy + rt + rr] : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < nr; ++rr) {
            const double y0 = ys[rr][ty], y1 = ys[rr][ty + 16];
#pragma unroll
            for (int v = 0; v < 6; ++v) {
                const double qv = qs[rr][tq + v];
                acc[0][v] = fma(qv, y0, acc[0][v]);
                acc[1][v] = fma(qv, y1, acc[1][v]);
            }
        }
        __syncthreads();
    }
    // partial[block][96][32]
    const int64_t pstride = (int64_t)kQC * kBmax;
    double* my = partial + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * pstride;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 6; ++v) my[(tq + v) * kBmax + ty + 16 * u] = acc[u][v];
    if (!last_block_arrived(&counters[blockIdx.y], gridDim.x)) return;
    for (int e = threadIdx.x; e < qn * b; e += 256) {
        const int c = e / b, yc = e % b;
        double s = 0.0;
        for (unsigned int bx = 0; bx < gridDim.x; ++bx)
            s += partial[((int64_t)blockIdx.y * gridDim.x + bx) * pstride + c * kBmax + yc];
        H[(int64_t)yc * ldh + q0 + c] = s;
    }
}

size_t gemm_tn_partial_elems(int64_t len, int q)
{
    const int64_t rb = len / 2048 + 1 < 512 ? len / 2048 + 1 : 512;
    return (size_t)rb * (size_t)((q + kQC - 1) / kQC) * kQC * kBmax;
}

void launch_gemm_tn(const double* Q, int64_t ldq, const double* Y, int64_t ldy, int64_t len, int q,
                    int b, double* H, int ldh, double* partial, unsigned int* counters,
                    hipStream_t s)
{
    if (q <= 0 || b <= 0) return;
    if (b > kBmax) fail(GKL_ERR_INVALID, "block width above 32");
    int64_t rb = len / 2048 + 1;
    if (rb > 512) rb = 512;
    const int64_t rpb = ((len + rb - 1) / rb + kTR - 1) / kTR * kTR;
    rb = (len + rpb - 1) / rpb;
    if (rb < 1) rb = 1;
    dim3 grid((unsigned int)rb, (unsigned int)((q + kQC - 1) / kQC));
    hipLaunchKernelGGL(gemm_tn_kernel, grid, dim3(256), 0, s, Q, ldq, Y, ldy, len, q, b, rpb, H,
                       ldh, partial, counters);
    GKL_LAUNCH_CHECK("gemm_tn_kernel");
}

// Y(len x b) -= Q(len x q) H(q x b); one row per thread, H in LDS.
__global__ void __launch_bounds__(256)
gemm_nn_sub_kernel(const double* __restrict__ Q, int64_t ldq, double* __restrict__ Y, int64_t ldy,
                   int64_t len, int q, int b, const double* __restrict__ H, int ldh)
{
    extern __shared__ double hs[];   // q x b
    for (int e = threadIdx.x; e < q * b; e += 256) hs[e] = H[(int64_t)(e / q) * ldh + (e % q)];
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= len) return;
    double acc[kBmax];
#pragma unroll
    for (int c = 0; c < kBmax; ++c) acc[c] = 0.0;
    for (int k = 0; k < q; ++k) {
        const double qv = Q[(int64_t)k * ldq + row];
#pragma unroll
        for (int c = 0; c < kBmax; ++c)
            if (c < b) acc[c] = fma(qv, hs[c * q + k], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < kBmax; ++c)
        if (c < b) Y[(int64_t)c * ldy + row] -= acc[c];
}

void launch_gemm_nn_sub(const double* Q, int64_t ldq, double* Y, int64_t ldy, int64_t len, int q,
                        int b, const double* H, int ldh, hipStream_t s)
{
    if (q <= 0 || b <= 0) return;
    hipLaunchKernelGGL(gemm_nn_sub_kernel, dim3(ceil_div(len, 256)), dim3(256),
                       sizeof(double) * (size_t)q * b, s, Q, ldq, Y, ldy, len, q, b, H, ldh);
    GKL_LAUNCH_CHECK("gemm_nn_sub_kernel");
}

// Cholesky of the b x b Gram matrix (column-major, ld b) in one workgroup, with an
// optional shift added to the diagonal; writes the upper factor Rn (G + shift I =
// Rn^T Rn), its inverse Ri, and R <- Rn R (accumulated; R = I on the first pass
// when first != 0).  Non-positive pivots are replaced by a tiny positive value and
// counted in *bad.
__global__ void chol_kernel(const double* __restrict__ Gm, int b, double shift_rel,
                            double* __restrict__ R, double* __restrict__ Ri, int first,
                            int* __restrict__ bad)
{
    __shared__ double A[kBmax][kBmax + 1];
    __shared__ double L[kBmax][kBmax + 1];      // upper factor Rn
    __shared__ double Iv[kBmax][kBmax + 1];     // inverse of Rn
    __shared__ double Rold[kBmax][kBmax + 1];
    const int t = threadIdx.x;
    for (int e = t; e < b * b; e += blockDim.x) {
        const int i = e % b, j = e / b;
        A[i][j] = Gm[e];
        Rold[i][j] = first ? (i == j ? 1.0 : 0.0) : R[e];
    }
    __syncthreads();
    if (t == 0) {
        double tr = 0.0;
        for (int i = 0; i < b; ++i) tr += A[i][i];
        const double sh = shift_rel * tr;
        for (int i = 0; i < b; ++i) A[i][i] += sh;
        // column Cholesky, upper factor: A = L^T L with L upper triangular
        for (int j = 0; j < b; ++j) {
            double d = A[j][j];
            for (int k = 0; k < j; ++k) d -= L[k][j] * L[k][j];
            if (!(d > 1e-300)) {
                d = 1e-300 + 1e-30 * (tr > 0 ? tr : 1.0);
                if (bad) *bad += 1;
            }
            const double l = sqrt(d);
            L[j][j] = l;
            for (int i = j + 1; i < b; ++i) {
                double s = A[j][i];
                for (int k = 0; k < j; ++k) s -= L[k][j] * L[k][i];
                L[j][i] = s / l;
            }
            for (int i = 0; i < j; ++i) L[j][i] = 0.0;
        }
        // inverse of the upper triangular L
        for (int j = b - 1; j >= 0; --j) {
            Iv[j][j] = 1.0 / L[j][j];
            for (int i = j - 1; i >= 0; --i) {
                double s = 0.0;
                for (int k = i + 1; k <= j; ++k) s += L[i][k] * Iv[k][j];
                Iv[i][j] = -s / L[i][i];
            }
            for (int i = j + 1; i < b; ++i) Iv[i][j] = 0.0;
        }
    }
    __syncthreads();
    for (int e = t; e < b * b; e += blockDim.x) {
        const int i = e % b, j = e / b;
        Ri[e] = Iv[i][j];
        double s = 0.0;
        for (int k = 0; k < b; ++k) s += L[i][k] * Rold[k][j];
        R[e] = s;
    }
}

// Y(len x b) <- Y Ri (Ri upper triangular b x b).
__global__ void __launch_bounds__(256)
trmm_right_kernel(double* __restrict__ Y, int64_t ldy, int64_t len, int b,
                  const double* __restrict__ Ri)
{
    __shared__ double rs[kBmax * kBmax];
    for (int e = threadIdx.x; e < b * b; e += 256) rs[e] = Ri[e];
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= len) return;
    double y[kBmax];
#pragma unroll
    for (int c = 0; c < kBmax; ++c) y[c] = c < b ? Y[(int64_t)c * ldy + row] : 0.0;
#pragma unroll
    for (int j = 0; j < kBmax; ++j) {
        if (j >= b) break;
        double s = 0.0;
        for (int k = 0; k <= j; ++k) s = fma(y[k], rs[j * b + k], s);
        Y[(int64_t)j * ldy + row] = s;
    }
}

// Shifted CholeskyQR3: Y (len x b) -> Q R with Q overwriting Y, R (b x b upper,
// column-major) written to Rout.  work: >= 3 b*b doubles.
void launch_block_qr(double* Y, int64_t ldy, int64_t len, int b, double* Rout, double* work,
                     double* partial, unsigned int* counters, int* bad, hipStream_t s)
{
    double* Gm = work;
    double* Ri = work + b * b;
    const double u = 1.1102230246251565e-16;
    const double shift = 11.0 * ((double)len * b + (double)b * (b + 1)) * u;
    for (int pass = 0; pass < 3; ++pass) {
        launch_gemm_tn(Y, ldy, Y, ldy, len, b, b, Gm, b, partial, counters, s);
        hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(64), 0, s, Gm, b, pass == 0 ? shift : 0.0,
                           Rout, Ri, pass == 0 ? 1 : 0, pass == 2 ? bad : nullptr);
        GKL_LAUNCH_CHECK("chol_kernel");
        hipLaunchKernelGGL(trmm_right_kernel, dim3(ceil_div(len, 256)), dim3(256), 0, s, Y, ldy,
                           len, b, Ri);
        GKL_LAUNCH_CHECK("trmm_right_kernel");
    }
}

// Block-bidiagonal projected matrix bookkeeping ------------------------------

// Write the b x b block X (column-major, ld b) into Bm (ldb) at (r0, c0); when
// transpose != 0 write X^T.
__global__ void put_block_kernel(double* __restrict__ Bm, int ldb, int r0, int c0,
                                 const double* __restrict__ X, int rows, int cols, int ldx,
                                 int transpose)
{
    for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) {
        const int i = e % rows, j = e / rows;
        Bm[(int64_t)(c0 + j) * ldb + r0 + i] = transpose ? X[(int64_t)i * ldx + j] : X[(int64_t)j * ldx + i];
    }
}

void launch_put_block(double* Bm, int ldb, int r0, int c0, const double* X, int rows, int cols,
                      int ldx, int transpose, hipStream_t s)
{
    hipLaunchKernelGGL(put_block_kernel, dim3(1), dim3(256), 0, s, Bm, ldb, r0, c0, X, rows, cols,
                       ldx, transpose);
    GKL_LAUNCH_CHECK("put_block_kernel");
}

// Copy the leading m x m of Bm (ldb) into a compact m x m buffer.
__global__ void copy_lead_kernel(const double* __restrict__ Bm, int ldb, int m,
                                 double* __restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)m * m;
         e += (int64_t)gridDim.x * blockDim.x)
        out[e] = Bm[(e / m) * ldb + (e % m)];
}

void launch_copy_lead(const double* Bm, int ldb, int m, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(copy_lead_kernel, dim3(ceil_div((int64_t)m * m, 256)), dim3(256), 0, s, Bm,
                       ldb, m, out);
    GKL_LAUNCH_CHECK("copy_lead_kernel");
}

// res_i = || C P(m-b:m, i) || for i < m (C upper b x b, column-major); nconv =
// leading i < k with res_i <= tol * S[0].
__global__ void block_residual_kernel(const double* __restrict__ C, int b,
                                      const double* __restrict__ P, int m,
                                      const double* __restrict__ S, int k, double tol,
                                      double* __restrict__ res, int* __restrict__ nconv)
{
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        double s2 = 0.0;
        for (int r = 0; r < b; ++r) {
            double v = 0.0;
            for (int c = r; c < b; ++c) v += C[c * b + r] * P[(int64_t)i * m + (m - b + c)];
            s2 += v * v;
        }
        res[i] = sqrt(s2);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nc = 0;
        for (int i = 0; i < k && i < m; ++i) {
            if (res[i] <= tol * S[0]) ++nc;
            else break;
        }
        *nconv = nc;
    }
}

void launch_block_residual(const double* C, int b, const double* P, int m, const double* S, int k,
                           double tol, double* res, int* nconv, hipStream_t s)
{
    hipLaunchKernelGGL(block_residual_kernel, dim3(1), dim3(256), 0, s, C, b, P, m, S, k, tol, res,
                       nconv);
    GKL_LAUNCH_CHECK("block_residual_kernel");
}

// After a restart: Bm := 0 in the leading (keep + b) square, diag(S[0:keep]), and
// the spike block Bm[0:keep, keep:keep+b] = (C P(m-b:m, 0:keep))^T.
__global__ void restart_block_kernel(double* __restrict__ Bm, int ldb, int keep, int b,
                                     const double* __restrict__ S, const double* __restrict__ C,
                                     const double* __restrict__ P, int m)
{
    const int tot = ldb;
    for (int64_t e = threadIdx.x; e < (int64_t)tot * tot; e += blockDim.x) Bm[e] = 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < keep; i += blockDim.x) {
        Bm[(int64_t)i * ldb + i] = S[i];
        for (int r = 0; r < b; ++r) {
            double v = 0.0;
            for (int c = r; c < b; ++c) v += C[c * b + r] * P[(int64_t)i * m + (m - b + c)];
            Bm[(int64_t)(keep + r) * ldb + i] = v;
        }
    }
}

void launch_restart_block(double* Bm, int ldb, int keep, int b, const double* S, const double* C,
                          const double* P, int m, hipStream_t s)
{
    hipLaunchKernelGGL(restart_block_kernel, dim3(1), dim3(1024), 0, s, Bm, ldb, keep, b, S, C, P,
                       m);
    GKL_LAUNCH_CHECK("restart_block_kernel");
}

}  // namespace gkl
