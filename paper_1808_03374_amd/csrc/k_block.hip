// FP64 block operations for block GKL bidiagonalisation (gfx950).
//
// Block Lanczos (named as future work in Section 5 of the paper) keeps the
// recurrence scalars, the Gram-Schmidt reorthogonalisation and the projected
// matrix in FP64; only the two products with the genotype matrix use the
// matrix-core path (split BF16 or int8 limbs).  This file holds the FP64 pieces:
//   * H = Q^T Y for tall Q (len x q) and Y (len x b) on the FP64 matrix cores:
//     one partial per workgroup, summed in a fixed order by a second kernel;
//   * Out -= Q H and Out = Q H (also in place, for Y <- Y R^-1), FP64 MFMA;
//   * block orthonormalisation by shifted Cholesky QR applied three times
//     (shifted CholeskyQR3, Fukaya, Kannan, Nakatsukasa, Yamamoto & Yanagisawa,
//     SIAM J. Sci. Comput. 2020): Gram matrix, Cholesky in one workgroup,
//     triangular solve applied to every row, R accumulated; a block whose
//     R falls below a guard level (a Krylov space running out on a matrix of
//     low rank) is re-orthogonalised column by column before R enters the
//     projected matrix;
//   * Ritz residuals of the block-bidiagonal projected matrix.
//
// v_mfma_f64_16x16x4f64 (one wave): lane l supplies A(l % 16, l / 16) and
// B(l / 16, l % 16); element e of the lane's result is D(l / 16 + 4 e, l % 16)
// (rows interleaved by four, unlike the FP32-output 16x16 forms).
// The contraction index may be permuted freely as long as A and B agree.
#include <math.h>

#include "kernels.h"

namespace gkl {

namespace {
constexpr int kBmax = 32;     // block width limit
constexpr int kTnQ = 64;      // Q columns per workgroup in Q^T Y (4 tiles of 16)
constexpr int kTnPart = kTnQ * kBmax;
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Rows per workgroup (a multiple of 128) and workgroup count for Q^T Y, at most
// max_wg workgroups per 64-column group (256 = one per CU; 1,024 measured no
// faster: the loads are column-strided, and the longer partial sums cost more
// than the extra workgroups saved).
constexpr int kTnWgMax = 256;
__host__ __device__ inline void tn_plan(int64_t len, int64_t* rows_per_wg, int* nwg,
                                        int max_wg = 256)
{
    int64_t r = (len + max_wg - 1) / max_wg;
    r = (r + 127) / 128 * 128;
    *rows_per_wg = r;
    *nwg = (int)((len + r - 1) / r);
}
}  // namespace

// Partial Q^T Y of one workgroup: rows [r0, r0 + rows_per_wg), Q columns [q0,
// q0 + 64).  Each wave walks steps of 32 rows; in a step, lane group g holds rows
// 8g .. 8g + 7 of its column and MFMA t contracts row 8g + t of every group.
// The four waves are summed through LDS in a fixed order.
__device__ __forceinline__ void tn_body(const double* __restrict__ Q, int64_t ldq,
                                        const double* __restrict__ Y, int64_t ldy, int64_t len,
                                        int q, int b, int64_t rows_per_wg, double* __restrict__ my,
                                        int bx, int by)
{
    __shared__ double red[2][kTnPart];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, g = lane >> 4;
    const int q0 = by * kTnQ;
    const int nqt = (q - q0 + 15) / 16 < 4 ? (q - q0 + 15) / 16 : 4;
    const int nbt = (b + 15) / 16;
    const int64_t r0 = (int64_t)bx * rows_per_wg;
    const int64_t r1 = r0 + rows_per_wg < len ? r0 + rows_per_wg : len;
    const double* qp[4];
    bool qok[4];
#pragma unroll
    for (int qt = 0; qt < 4; ++qt) {
        const int c = q0 + qt * 16 + col;
        qok[qt] = c < q;
        qp[qt] = Q + (int64_t)(qok[qt] ? c : 0) * ldq;
    }
    const double* yp[2];
    bool yok[2];
#pragma unroll
    for (int bt = 0; bt < 2; ++bt) {
        const int c = bt * 16 + col;
        yok[bt] = c < b;
        yp[bt] = Y + (int64_t)(yok[bt] ? c : 0) * ldy;
    }
    v4d acc[4][2];
#pragma unroll
    for (int qt = 0; qt < 4; ++qt)
#pragma unroll
        for (int bt = 0; bt < 2; ++bt) acc[qt][bt] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int64_t rs = r0 + wave * 32; rs < r1; rs += 128) {
        const int64_t rb = rs + 8 * g;
        double qv[4][8], yv[2][8];
        const bool full = rb + 8 <= r1;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bool ok = full || rb + t < r1;
#pragma unroll
            for (int bt = 0; bt < 2; ++bt) yv[bt][t] = (ok && yok[bt]) ? yp[bt][rb + t] : 0.0;
#pragma unroll
            for (int qt = 0; qt < 4; ++qt) qv[qt][t] = (ok && qok[qt]) ? qp[qt][rb + t] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int qt = 0; qt < 4; ++qt) {
                if (qt >= nqt) continue;
                acc[qt][0] = mfma64(qv[qt][t], yv[0][t], acc[qt][0]);
                if (nbt > 1) acc[qt][1] = mfma64(qv[qt][t], yv[1][t], acc[qt][1]);
            }
    }
    // lane's element e of tile (qt, bt) is H(q0 + qt*16 + g + 4e, bt*16 + col)
    if (wave < 2) {
#pragma unroll
        for (int qt = 0; qt < 4; ++qt)
#pragma unroll
            for (int bt = 0; bt < 2; ++bt)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    red[wave][(qt * 16 + g + 4 * e) * kBmax + bt * 16 + col] = acc[qt][bt][e];
    }
    __syncthreads();
    if (wave >= 2) {
#pragma unroll
        for (int qt = 0; qt < 4; ++qt)
#pragma unroll
            for (int bt = 0; bt < 2; ++bt)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    red[wave - 2][(qt * 16 + g + 4 * e) * kBmax + bt * 16 + col] += acc[qt][bt][e];
    }
    __syncthreads();
    // only the b live columns of each of the 64 rows are ever read
    for (int e = threadIdx.x; e < kTnQ * b; e += 256) {
        const int idx = (e / b) * kBmax + e % b;
        my[idx] = red[0][idx] + red[1][idx];
    }
}

__global__ void __launch_bounds__(256)
gemm_tn_kernel(const double* __restrict__ Q, int64_t ldq, const double* __restrict__ Y,
               int64_t ldy, int64_t len, int q, int b, int64_t rows_per_wg,
               double* __restrict__ partial, const int* __restrict__ enable,
               const int* __restrict__ skip)
{
    if ((enable && *enable == 0) || (skip && *skip)) return;   // the same for every thread
    tn_body(Q, ldq, Y, ldy, len, q, b, rows_per_wg,
            partial + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * kTnPart, blockIdx.x,
            blockIdx.y);
}

// H(qc, j) = sum over workgroups of the partials: 16 lanes per output, lane r
// adding workgroups r, r + 16, ... in order, then a fixed butterfly.
__global__ void __launch_bounds__(256)
gemm_tn_reduce_kernel(const double* __restrict__ partial, int nwg, int q, int b,
                      double* __restrict__ H, int ldh, const int* __restrict__ enable,
                      const int* __restrict__ skip)
{
    if ((enable && *enable == 0) || (skip && *skip)) return;
    const int t = blockIdx.x * 16 + (threadIdx.x >> 4);
    const int r = threadIdx.x & 15;
    const bool live = t < q * b;
    const int qc = live ? t / b : 0, j = live ? t % b : 0;
    const double* src =
        partial + (int64_t)(qc / kTnQ) * nwg * kTnPart + (qc % kTnQ) * kBmax + j;
    double s = 0.0;
    if (live)
        for (int x = r; x < nwg; x += 16) s += src[(int64_t)x * kTnPart];
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) s += __shfl_xor(s, off, 16);
    if (live && r == 0) H[(int64_t)j * ldh + qc] = s;
}

// Partial buffer for any len: the single-context plan uses at most kTnWgMax
// workgroups per column group.
size_t gemm_tn_partial_elems(int64_t, int q)
{
    return (size_t)kTnWgMax * (size_t)ceil_div(q < 1 ? 1 : q, kTnQ) * kTnPart;
}

void launch_gemm_tn(const double* Q, int64_t ldq, const double* Y, int64_t ldy, int64_t len, int q,
                    int b, double* H, int ldh, double* partial, hipStream_t s)
{
    launch_gemm_tn_gated(Q, ldq, Y, ldy, len, q, b, H, ldh, partial, nullptr, nullptr, s);
}

void launch_gemm_tn_gated(const double* Q, int64_t ldq, const double* Y, int64_t ldy, int64_t len,
                          int q, int b, double* H, int ldh, double* partial, const int* enable,
                          const int* skip, hipStream_t s)
{
    if (q <= 0 || b <= 0 || len <= 0) return;
    if (b > kBmax) fail(GKL_ERR_INVALID, "block width above 32");
    int64_t rpw;
    int nwg;
    tn_plan(len, &rpw, &nwg, kTnWgMax);
    if (nwg > kTnWgMax) fail(GKL_ERR_INTERNAL, "gemm_tn plan exceeds its partial buffer");
    dim3 grid((unsigned int)nwg, (unsigned int)ceil_div(q, kTnQ));
    hipLaunchKernelGGL(gemm_tn_kernel, grid, dim3(256), 0, s, Q, ldq, Y, ldy, len, q, b, rpw,
                       partial, enable, skip);
    GKL_LAUNCH_CHECK("gemm_tn_kernel");
    hipLaunchKernelGGL(gemm_tn_reduce_kernel, dim3(ceil_div(q * b, 16)), dim3(256), 0, s, partial,
                       nwg, q, b, H, ldh, enable, skip);
    GKL_LAUNCH_CHECK("gemm_tn_reduce_kernel");
}

// Out(len x nc) = Q(len x q) H(q x nc)  (subtract == 0), or Out -= Q H.  Each wave
// owns 64 rows (four row tiles) and 32 output columns (grid.y covers more); the
// contraction runs over q in steps of 4.  Q and Out may be the same matrix when
// nc <= 32: a wave reads all of its rows before it writes them.
__global__ void __launch_bounds__(256)
gemm_nn_kernel(const double* Q, int64_t ldq, int q, const double* __restrict__ H, int ldh,
               double* Out, int64_t ldo, int64_t len, int nc, int subtract)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, g = lane >> 4;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * 64;
    if (r0 >= len) return;
    const int c0 = blockIdx.y * 32;
    const int nbt = nc - c0 > 16 ? 2 : 1;
    bool rok[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) rok[rt] = r0 + rt * 16 + col < len;
    bool hok[2];
    int hc[2];
#pragma unroll
    for (int bt = 0; bt < 2; ++bt) {
        hc[bt] = c0 + bt * 16 + col;
        hok[bt] = hc[bt] < nc;
        if (!hok[bt]) hc[bt] = 0;
    }
    v4d acc[4][2];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int bt = 0; bt < 2; ++bt) acc[rt][bt] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < q; k += 4) {
        const int kk = k + g;
        const bool kok = kk < q;
        const double* qc = Q + (int64_t)(kok ? kk : 0) * ldq + r0 + col;
        double a[4], hb[2];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) a[rt] = (kok && rok[rt]) ? qc[rt * 16] : 0.0;
#pragma unroll
        for (int bt = 0; bt < 2; ++bt)
            hb[bt] = (kok && hok[bt]) ? H[(int64_t)hc[bt] * ldh + kk] : 0.0;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            acc[rt][0] = mfma64(a[rt], hb[0], acc[rt][0]);
            if (nbt > 1) acc[rt][1] = mfma64(a[rt], hb[1], acc[rt][1]);
        }
    }
    // element e of tile (rt, bt): Out(r0 + rt*16 + g + 4e, c0 + bt*16 + col)
#pragma unroll
    for (int bt = 0; bt < 2; ++bt) {
        const int c = c0 + bt * 16 + col;
        if (c >= nc) continue;
        double* oc = Out + (int64_t)c * ldo;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = r0 + rt * 16 + g + 4 * e;
                if (row < len) oc[row] = subtract ? oc[row] - acc[rt][bt][e] : acc[rt][bt][e];
            }
    }
}

void launch_gemm_nn(const double* Q, int64_t ldq, int q, const double* H, int ldh, double* Out,
                    int64_t ldo, int64_t len, int nc, int subtract, hipStream_t s)
{
    if (nc <= 0 || len <= 0) return;
    if (q <= 0) {
        if (subtract) return;
        fail(GKL_ERR_INTERNAL, "gemm_nn with an empty contraction");
    }
    if ((const double*)Out == Q && nc > 32)
        fail(GKL_ERR_INTERNAL, "in-place gemm_nn needs at most 32 output columns");
    dim3 grid((unsigned int)ceil_div(len, (int64_t)256), (unsigned int)ceil_div(nc, 32));
    hipLaunchKernelGGL(gemm_nn_kernel, grid, dim3(256), 0, s, Q, ldq, q, H, ldh, Out, ldo, len, nc,
                       subtract);
    GKL_LAUNCH_CHECK("gemm_nn_kernel");
}

void launch_gemm_nn_sub(const double* Q, int64_t ldq, double* Y, int64_t ldy, int64_t len, int q,
                        int b, const double* H, int ldh, hipStream_t s)
{
    launch_gemm_nn(Q, ldq, q, H, ldh, Y, ldy, len, b, 1, s);
}

// ---------------------------------------------------------------------------
// Batched projections h = Q^T r of every active problem (grid.z = problem)
// ---------------------------------------------------------------------------
size_t batch_tn_partial_elems(int hstride)
{
    return (size_t)256 * (size_t)ceil_div(hstride, kTnQ) * kTnPart;
}

namespace {
struct ProjSide {
    int64_t len;
    int ncols;
    const double* Q;
    const double* r;
};
__device__ __forceinline__ ProjSide proj_side(const BatchDesc& D, int j, int side)
{
    ProjSide s;
    if (side == 0) {
        s.len = D.n;
        s.ncols = j;
        s.Q = D.U;
        s.r = D.U + (int64_t)j * D.n;
    } else {
        s.len = D.p;
        s.ncols = j + 1;
        s.Q = D.V;
        s.r = D.V + (int64_t)(j + 1) * D.p;
    }
    return s;
}
}  // namespace

// Partials of one problem live at tnpart + (chunk * 256 + workgroup) * kTnPart.
__global__ void __launch_bounds__(256)
batch_tn_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state, int side)
{
    const BatchDesc& D = desc[blockIdx.z];
    if (!*D.active) return;
    const ProjSide S = proj_side(D, state[0], side);
    int64_t rpw;
    int nwg;
    tn_plan(S.len, &rpw, &nwg);
    if ((int)blockIdx.x >= nwg || (int)blockIdx.y * kTnQ >= S.ncols) return;   // whole workgroup
    tn_body(S.Q, S.len, S.r, S.len, S.len, S.ncols, 1, rpw,
            D.tnpart + ((int64_t)blockIdx.y * 256 + blockIdx.x) * kTnPart, blockIdx.x, blockIdx.y);
}

// h[c] = sum of the problem's workgroup partials, 16 lanes per column.
__global__ void __launch_bounds__(256)
batch_tn_reduce_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state, int side)
{
    const BatchDesc& D = desc[blockIdx.y];
    if (!*D.active) return;
    const ProjSide S = proj_side(D, state[0], side);
    int64_t rpw;
    int nwg;
    tn_plan(S.len, &rpw, &nwg);
    const int t = blockIdx.x * 16 + (threadIdx.x >> 4);
    const int r = threadIdx.x & 15;
    const bool live = t < S.ncols;
    const double* src =
        D.tnpart + (int64_t)(live ? t / kTnQ : 0) * 256 * kTnPart + (live ? t % kTnQ : 0) * kBmax;
    double s = 0.0;
    if (live)
        for (int x = r; x < nwg; x += 16) s += src[(int64_t)x * kTnPart];
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) s += __shfl_xor(s, off, 16);
    if (live && r == 0) D.h[t] = s;
}

void launch_batch_proj(const BatchDesc* d, const int* state, int count, int side, int hstride,
                       hipStream_t s)
{
    hipLaunchKernelGGL(batch_tn_kernel, dim3(256, ceil_div(hstride, kTnQ), count), dim3(256), 0, s,
                       d, state, side);
    GKL_LAUNCH_CHECK("batch_tn_kernel");
    hipLaunchKernelGGL(batch_tn_reduce_kernel, dim3(ceil_div(hstride, 16), count), dim3(256), 0, s,
                       d, state, side);
    GKL_LAUNCH_CHECK("batch_tn_reduce_kernel");
}

// Cholesky of the b x b Gram matrix (column-major, ld b) in one workgroup, with an
// optional shift (shift_rel times the trace) added to the diagonal; writes the
// upper factor Rn (G + shift I = Rn^T Rn), its inverse Ri, and R <- Rn R
// (accumulated; R = I on the first pass when first != 0).  Non-positive pivots
// are replaced by a tiny positive value and counted in *bad.  Right-looking
// factorisation and a row-oriented back substitution, one barrier per stage.
//
// guard (optional, per solve): guard[0] is the running maximum of the squared
// column norms the first pass has seen (a scale of the largest singular value);
// the last pass (pass == 2) sets guard[1] to 1 when a diagonal entry of the
// accumulated R is at most kGuardRel times that scale, else to 0.  Such a column
// was (numerically) dependent on the basis or on the block's earlier columns:
// the Cholesky QR scales its rounding residue up to unit length, and that
// residue is not orthogonal to the basis.  block_finish_kernel repairs it.
constexpr double kGuardRel = 1e-4;

__device__ __forceinline__ void chol_body(const double* Gm, int b, double shift_rel,
                                          double* __restrict__ R, double* __restrict__ Ri,
                                          int first, int* __restrict__ bad,
                                          double* __restrict__ guard, int pass)
{
    __shared__ double A[kBmax][kBmax + 1];      // becomes the upper factor Rn
    __shared__ double Xr[kBmax][kBmax + 1];     // inverse of Rn
    __shared__ double Rold[kBmax][kBmax + 1];
    __shared__ double trace;
    __shared__ int nbad;
    const int t = threadIdx.x;
    for (int e = t; e < b * b; e += blockDim.x) {
        const int i = e % b, j = e / b;
        A[i][j] = Gm[e];
        Rold[i][j] = first ? (i == j ? 1.0 : 0.0) : R[e];
        Xr[i][j] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    if (t == 0) {
        double tr = 0.0;
        for (int i = 0; i < b; ++i) tr += A[i][i];
        trace = tr;
        nbad = 0;
        if (guard && pass == 0) {
            double mx = guard[0];
            for (int i = 0; i < b; ++i) mx = fmax(mx, A[i][i]);
            guard[0] = mx;
        }
        const double sh = shift_rel * tr;
        for (int i = 0; i < b; ++i) A[i][i] += sh;
    }
    __syncthreads();
    for (int j = 0; j < b; ++j) {
        if (t == 0) {
            double d = A[j][j];
            if (!(d > 1e-300)) {
                d = 1e-300 + 1e-30 * (trace > 0 ? trace : 1.0);
                ++nbad;
            }
            A[j][j] = sqrt(d);
        }
        __syncthreads();
        const double l = A[j][j];
        for (int i = j + 1 + t; i < b; i += blockDim.x) A[j][i] /= l;
        __syncthreads();
        const int w = b - j - 1;
        for (int e = t; e < w * w; e += blockDim.x) {
            const int i = j + 1 + e / w, i2 = j + 1 + e % w;
            A[i][i2] -= A[j][i] * A[j][i2];
        }
        __syncthreads();
    }
    for (int e = t; e < b * b; e += blockDim.x) {
        const int i = e % b, j = e / b;
        if (i > j) A[i][j] = 0.0;
    }
    __syncthreads();
    // Rn X = I, X upper: rows from the bottom, each finished row updating those above
    for (int i = b - 1; i >= 0; --i) {
        const double d = A[i][i];
        for (int j = i + t; j < b; j += blockDim.x) Xr[i][j] /= d;
        __syncthreads();
        const int w = b - i;
        for (int e = t; e < i * w; e += blockDim.x) {
            const int k = e / w, j = i + e % w;
            Xr[k][j] -= A[k][i] * Xr[i][j];
        }
        __syncthreads();
    }
    for (int e = t; e < b * b; e += blockDim.x) {
        const int i = e % b, j = e / b;
        Ri[e] = j >= i ? Xr[i][j] : 0.0;
        double s = 0.0;
        for (int k = i; k < b; ++k) s += A[i][k] * Rold[k][j];
        R[e] = s;
    }
    if (t == 0 && bad && nbad) *bad += nbad;
    if (t == 0 && guard && pass == 2) {
        const double floor = kGuardRel * sqrt(guard[0]);
        int weak = 0;
        for (int j = 0; j < b; ++j) weak |= A[j][j] * Rold[j][j] <= floor ? 1 : 0;
        guard[1] = weak ? 1.0 : 0.0;
    }
}

__global__ void __launch_bounds__(256)
chol_kernel(const double* __restrict__ Gm, int b, double shift_rel, double* __restrict__ R,
            double* __restrict__ Ri, int first, int* __restrict__ bad, double* __restrict__ guard,
            int pass)
{
    chol_body(Gm, b, shift_rel, R, Ri, first, bad, guard, pass);
}

// Blocks of kB <= 4 columns, one row per thread (grid-stride): with apply, the
// row is first multiplied by the previous pass's inverse factor (upper
// triangular, column-major in Ri) and written back; with partial, the
// workgroup's sums of y_i y_j (i <= j, kB (kB + 1) / 2 of them) go to
// partial[wg * kG + e].  One pass over Y serves both halves of a CholeskyQR
// step, where the general path reads Y column-strided twice.
template <int kB>
__global__ void __launch_bounds__(256)
gram_rows_kernel(double* __restrict__ Y, int64_t ldy, int64_t len, const double* __restrict__ Ri,
                 int apply, double* __restrict__ partial)
{
    constexpr int kG = kB * (kB + 1) / 2;
    __shared__ double ri[kB * kB];
    __shared__ double red[4][kG];
    if (apply)
        for (int e = threadIdx.x; e < kB * kB; e += blockDim.x) ri[e] = Ri[e];
    __syncthreads();
    double g[kG];
#pragma unroll
    for (int e = 0; e < kG; ++e) g[e] = 0.0;
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < len;
         row += (int64_t)gridDim.x * blockDim.x) {
        double y[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) y[j] = Y[(int64_t)j * ldy + row];
        if (apply) {
            double z[kB];
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                double a = 0.0;
#pragma unroll
                for (int i = 0; i <= j; ++i) a = fma(y[i], ri[i + j * kB], a);
                z[j] = a;
            }
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                Y[(int64_t)j * ldy + row] = z[j];
                y[j] = z[j];
            }
        }
        int e = 0;
#pragma unroll
        for (int i = 0; i < kB; ++i)
#pragma unroll
            for (int j = i; j < kB; ++j) {
                g[e] = fma(y[i], y[j], g[e]);
                ++e;
            }
    }
    if (!partial) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < kG; ++e) {
        const double v = wave_sum(g[e]);
        if (lane == 0) red[wave][e] = v;
    }
    __syncthreads();
    if (threadIdx.x < kG)
        partial[(int64_t)blockIdx.x * kG + threadIdx.x] =
            ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// The Gram matrix from gram_rows_kernel's nwg partials (one wave per entry,
// lanes adding workgroups in order, then a fixed butterfly), then the Cholesky
// step of chol_kernel.
template <int kB>
__global__ void __launch_bounds__(256)
gram_chol_kernel(const double* __restrict__ partial, int nwg, double shift_rel,
                 double* __restrict__ R, double* __restrict__ Ri, int first, int* __restrict__ bad,
                 double* __restrict__ guard, int pass)
{
    constexpr int kG = kB * (kB + 1) / 2;
    __shared__ double Gs[kB * kB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = wave; e < kG; e += (int)(blockDim.x >> 6)) {
        double sum = 0.0;
        for (int w = lane; w < nwg; w += 64) sum += partial[(int64_t)w * kG + e];
        sum = wave_sum(sum);
        if (lane == 0) {
            int i = 0, r = e;          // entry e is (i, j), i <= j, rows of the upper triangle
            while (r >= kB - i) {
                r -= kB - i;
                ++i;
            }
            const int j = i + r;
            Gs[i + j * kB] = sum;
            Gs[j + i * kB] = sum;
        }
    }
    __syncthreads();
    chol_body(Gs, kB, shift_rel, R, Ri, first, bad, guard, pass);
}

template <int kB>
static void small_block_qr(double* Y, int64_t ldy, int64_t len, double* Rout, double* Ri,
                           double* partial, int* bad, double shift, double* guard, hipStream_t s)
{
    int64_t g = ceil_div(len, 256);
    const int nwg = (int)(g < 1024 ? g : 1024);
    for (int pass = 0; pass < 3; ++pass) {
        hipLaunchKernelGGL(gram_rows_kernel<kB>, dim3(nwg), dim3(256), 0, s, Y, ldy, len, Ri,
                           pass > 0 ? 1 : 0, partial);
        GKL_LAUNCH_CHECK("gram_rows_kernel");
        hipLaunchKernelGGL(gram_chol_kernel<kB>, dim3(1), dim3(256), 0, s, partial, nwg,
                           pass == 0 ? shift : 0.0, Rout, Ri, pass == 0 ? 1 : 0,
                           pass == 2 ? bad : nullptr, guard, pass);
        GKL_LAUNCH_CHECK("gram_chol_kernel");
    }
    hipLaunchKernelGGL(gram_rows_kernel<kB>, dim3(nwg), dim3(256), 0, s, Y, ldy, len, Ri, 1,
                       nullptr);
    GKL_LAUNCH_CHECK("gram_rows_kernel");
}

// Shifted CholeskyQR3: Y (len x b) -> Q R with Q overwriting Y, R (b x b upper,
// column-major) written to Rout.  work: >= 3 b*b doubles.
void launch_block_qr(double* Y, int64_t ldy, int64_t len, int b, double* Rout, double* work,
                     double* partial, int* bad, hipStream_t s, double* guard)
{
    double* Gm = work;
    double* Ri = work + b * b;
    const double u = 1.1102230246251565e-16;
    const double shift = 11.0 * ((double)len * b + (double)b * (b + 1)) * u;
    switch (b) {   // up to four columns: the row-parallel passes (7 launches instead of 12)
    case 1: small_block_qr<1>(Y, ldy, len, Rout, Ri, partial, bad, shift, guard, s); return;
    case 2: small_block_qr<2>(Y, ldy, len, Rout, Ri, partial, bad, shift, guard, s); return;
    case 3: small_block_qr<3>(Y, ldy, len, Rout, Ri, partial, bad, shift, guard, s); return;
    case 4: small_block_qr<4>(Y, ldy, len, Rout, Ri, partial, bad, shift, guard, s); return;
    default: break;
    }
    for (int pass = 0; pass < 3; ++pass) {
        launch_gemm_tn(Y, ldy, Y, ldy, len, b, b, Gm, b, partial, s);
        hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(256), 0, s, Gm, b, pass == 0 ? shift : 0.0,
                           Rout, Ri, pass == 0 ? 1 : 0, pass == 2 ? bad : nullptr, guard, pass);
        GKL_LAUNCH_CHECK("chol_kernel");
        launch_gemm_nn(Y, ldy, b, Ri, b, Y, ldy, len, b, 0, s);
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

// After the block QR of Y (len x b, Y = Q R with Q in place): when the QR set
// guard[1] (a column of R below the guard level), re-orthogonalise Q column by
// column against the basis Qb (len x q) and the block's earlier columns, with a
// second and third pass while a pass shrinks the column below 1/sqrt(2) of its
// length (Kahan's criterion for Gram-Schmidt).  A column still shrinking after
// three passes lies in the span and becomes zero.  With Q = Q' T (T upper
// triangular: the block coefficients above the diagonal, the final lengths on
// it; basis components, which are rounding residue, are dropped), R becomes
// T R.  Then R (or R^T when transpose != 0) is written into Bm at (r0, c0).
// One workgroup: the repair is rare (a Krylov space that runs out on a matrix
// of low rank), the write is every step's.
constexpr int kRepChunk = 256;

__global__ void __launch_bounds__(1024)
block_finish_kernel(double* __restrict__ Y, int64_t ldy, int64_t len, int b,
                    const double* __restrict__ Qb, int64_t ldq, int q, double* __restrict__ R,
                    const double* __restrict__ guard, double* __restrict__ Bm, int ldb, int r0,
                    int c0, int transpose)
{
    __shared__ double T[kBmax][kBmax + 1];
    __shared__ double Rs[kBmax][kBmax + 1];
    __shared__ double coef[kRepChunk];
    __shared__ double red[16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = (int)(blockDim.x >> 6);
    for (int e = t; e < b * b; e += blockDim.x) Rs[e % b][e / b] = R[e];
    const bool repair = guard && guard[1] != 0.0;
    if (repair) {
        for (int e = t; e < b * b; e += blockDim.x) T[e % b][e / b] = 0.0;
        __syncthreads();
        for (int j = 0; j < b; ++j) {
            double* w = Y + (int64_t)j * ldy;
            double a = 0.0;
            for (int64_t i = t; i < len; i += blockDim.x) a = fma(w[i], w[i], a);
            double before = sqrt(block_sum(a, red));
            double nu = before;
            bool accepted = false;
            for (int pass = 0; pass < 3 && !accepted; ++pass) {
                const int ncol = q + j;     // basis, then the block's repaired columns
                for (int cb = 0; cb < ncol; cb += kRepChunk) {
                    const int cn = ncol - cb < kRepChunk ? ncol - cb : kRepChunk;
                    for (int c = wave; c < cn; c += nw) {
                        const int col = cb + c;
                        const double* x = col < q ? Qb + (int64_t)col * ldq : Y + (int64_t)(col - q) * ldy;
                        double d = 0.0;
                        for (int64_t i = lane; i < len; i += 64) d = fma(x[i], w[i], d);
                        d = wave_sum(d);
                        if (lane == 0) coef[c] = d;
                    }
                    __syncthreads();
                    for (int64_t i = t; i < len; i += blockDim.x) {
                        double v = w[i];
                        for (int c = 0; c < cn; ++c) {
                            const int col = cb + c;
                            const double* x = col < q ? Qb + (int64_t)col * ldq
                                                      : Y + (int64_t)(col - q) * ldy;
                            v = fma(-coef[c], x[i], v);
                        }
                        w[i] = v;
                    }
                    if (t < cn && cb + t >= q) T[cb + t - q][j] += coef[t];
                    __syncthreads();
                }
                a = 0.0;
                for (int64_t i = t; i < len; i += blockDim.x) a = fma(w[i], w[i], a);
                nu = sqrt(block_sum(a, red));
                accepted = nu > 0.70710678118654752 * before;
                before = nu;
            }
            const double scale = accepted && nu > 0.0 ? 1.0 / nu : 0.0;
            for (int64_t i = t; i < len; i += blockDim.x) w[i] *= scale;
            if (t == 0) T[j][j] = scale != 0.0 ? nu : 0.0;
            __syncthreads();
        }
        // R <- T R (both upper triangular), kept in Rs
        double v[4];
        int cnt = 0;
        for (int e = t; e < b * b && cnt < 4; e += blockDim.x, ++cnt) {
            const int i = e % b, k = e / b;
            double s = 0.0;
            for (int l = i; l <= k; ++l) s += T[i][l] * Rs[l][k];
            v[cnt] = i <= k ? s : 0.0;
        }
        __syncthreads();
        cnt = 0;
        for (int e = t; e < b * b && cnt < 4; e += blockDim.x, ++cnt) {
            Rs[e % b][e / b] = v[cnt];
            R[e] = v[cnt];
        }
    }
    __syncthreads();
    for (int e = t; e < b * b; e += blockDim.x) {
        const int i = e % b, j = e / b;
        Bm[(int64_t)(c0 + j) * ldb + r0 + i] = transpose ? Rs[j][i] : Rs[i][j];
    }
}

void launch_block_finish(double* Y, int64_t ldy, int64_t len, int b, const double* Qb,
                         int64_t ldq, int q, double* R, const double* guard, double* Bm, int ldb,
                         int r0, int c0, int transpose, hipStream_t s)
{
    hipLaunchKernelGGL(block_finish_kernel, dim3(1), dim3(1024), 0, s, Y, ldy, len, b, Qb, ldq, q,
                       R, guard, Bm, ldb, r0, c0, transpose);
    GKL_LAUNCH_CHECK("block_finish_kernel");
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
