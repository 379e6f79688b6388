// Gram-Schmidt reorthogonalisation, normalisation and the small dense products
// on the Krylov bases (gfx950, FP64).
//
// Section 3 of the paper, "Choice of reorthogonalization strategy": full
// reorthogonalisation uses classical Gram-Schmidt applied twice (CGS2); the
// second pass may be skipped adaptively when the first pass lost few digits
// (criterion of Daniel, Gragg, Kaufman & Stewart: keep the result when its norm
// is at least 1/sqrt(2) of the norm before the pass).
//
// The bases are column-major (length x columns), so every pass streams
// contiguous rows.  The projection h = Q^T r runs on the FP64 matrix cores (the
// tall-skinny Q^T Y kernel with one vector); norms are two-stage reductions with
// a fixed order (block partials, then the last block to arrive sums them).  All
// results are deterministic.
#include <math.h>

#include "engine.h"

namespace gkl {

namespace {
constexpr int kOT = 256;      // threads per block
constexpr int kNR = 4;        // norm / update: rows per thread
constexpr int kNRows = kOT * kNR;
}  // namespace

size_t ortho_partial_elems(int64_t len, int)
{
    return (size_t)ceil_div(len, kNRows) + 1;   // norm partials (projections use tn_partial)
}

// r <- r - Q h (all columns).  With npart != NULL each block also writes the sum
// of squares of its updated rows to npart[block] (the norm that follows needs no
// second pass over r), and block 0 adds 2 to *passes when passes != NULL.
__global__ void __launch_bounds__(kOT)
update_kernel(const double* __restrict__ Q, int64_t ldq, int64_t len, int ncols,
              double* __restrict__ r, const double* __restrict__ h, const int* __restrict__ enable,
              const int* __restrict__ skip, double* __restrict__ npart, int* __restrict__ passes)
{
    if (enable && *enable == 0) return;
    if (skip && *skip) return;
    extern __shared__ double hs[];
    __shared__ double red[16];
    for (int c = threadIdx.x; c < ncols; c += kOT) hs[c] = h[c];
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * kOT + threadIdx.x;
    double a = 0.0;
    if (row < len) {
        a = r[row];
        int c = 0;
        for (; c + 8 <= ncols; c += 8) {
            double q[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) q[t] = Q[(int64_t)(c + t) * ldq + row];
#pragma unroll
            for (int t = 0; t < 8; ++t) a = fma(-q[t], hs[c + t], a);
        }
        for (; c < ncols; ++c) a = fma(-Q[(int64_t)c * ldq + row], hs[c], a);
        r[row] = a;
    }
    if (npart) {
        const double ss = block_sum(a * a, red);
        if (threadIdx.x == 0) npart[blockIdx.x] = ss;
    }
    if (passes && blockIdx.x == 0 && threadIdx.x == 0) *passes += 2;
}

// ||r||^2 by blocks, the last block finishes: nrm = sqrt; breakdown test against
// eps * max(norm_est, nrm) * root_maxdim; writes *nrm_out (0 on breakdown), the
// flag, and updates norm_est.  With decide == 0 it only writes sqrt into nrm_out.
__global__ void __launch_bounds__(kOT)
norm_kernel(const double* __restrict__ r, int64_t len, double* __restrict__ nrm_out,
            double* __restrict__ norm_est, double root_maxdim, int* __restrict__ flag,
            int* __restrict__ first_breakdown, int step, int decide, double* __restrict__ partial,
            unsigned int* __restrict__ counter)
{
    __shared__ double sh[16];
    double a = 0.0;
#pragma unroll
    for (int t = 0; t < kNR; ++t) {
        const int64_t row = (int64_t)blockIdx.x * kNRows + t * kOT + threadIdx.x;
        if (row < len) {
            const double x = r[row];
            a = fma(x, x, a);
        }
    }
    a = block_sum(a, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = a;
    if (!last_block_arrived(counter, gridDim.x)) return;
    double t2 = 0.0;
    for (unsigned int b = threadIdx.x; b < gridDim.x; b += kOT) t2 += partial[b];
    t2 = block_sum(t2, sh);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(t2);
        if (!decide) {
            *nrm_out = nrm;
            return;
        }
        double est = *norm_est;
        if (nrm > est) est = nrm;
        const double thresh = 2.220446049250313e-16 * est * root_maxdim;
        if (nrm <= thresh) {
            *nrm_out = 0.0;
            *flag = 1;
            if (first_breakdown && *first_breakdown < 0) *first_breakdown = step;
        } else {
            *nrm_out = nrm;
            *flag = 0;
        }
        *norm_est = est;
    }
}

static void launch_update(const double* Q, int64_t ldq, int64_t len, int ncols, double* r,
                          const double* h, const int* enable, const int* skip, hipStream_t s,
                          double* npart = nullptr, int* passes = nullptr)
{
    hipLaunchKernelGGL(update_kernel, dim3(ceil_div(len, kOT)), dim3(kOT),
                       sizeof(double) * (size_t)ncols, s, Q, ldq, len, ncols, r, h, enable, skip,
                       npart, passes);
    GKL_LAUNCH_CHECK("update_kernel");
}

__global__ void adapt_decide_kernel(const double* __restrict__ n0, const double* __restrict__ n1,
                                    int* __restrict__ skip, int* __restrict__ passes,
                                    const int* __restrict__ enable)
{
    if (enable && *enable == 0) return;
    const int sk = (*n1) >= 0.7071067811865476 * (*n0) ? 1 : 0;
    *skip = sk;
    if (passes) *passes += sk ? 1 : 2;
}

void launch_norm_raw(const double* r, int64_t len, double* out, OrthoWork& w, hipStream_t s)
{
    hipLaunchKernelGGL(norm_kernel, dim3(ceil_div(len, kNRows)), dim3(kOT), 0, s, r, len, out,
                       nullptr, 1.0, nullptr, nullptr, 0, 0, w.partial, w.counters + 1);
    GKL_LAUNCH_CHECK("norm_kernel");
}

void launch_cgs2(const double* Q, int64_t ldq, int64_t len, int ncols, double* r,
                 const int* enable, int adaptive, int* passes, OrthoWork& w, hipStream_t s)
{
    if (ncols <= 0) return;
    double* h1 = w.h;
    double* n0 = w.h + (ncols + 1);
    double* n1 = n0 + 1;
    int* skip = reinterpret_cast<int*>(n0 + 2);
    // h = Q^T r on the FP64 matrix cores (one column of the 16-wide B operand used)
    auto proj = [&](const int* sk) {
        launch_gemm_tn_gated(Q, ldq, r, len, len, ncols, 1, h1, ncols, w.tn_partial, enable, sk, s);
    };
    if (adaptive) {
        launch_norm_raw(r, len, n0, w, s);
        proj(nullptr);
        launch_update(Q, ldq, len, ncols, r, h1, enable, nullptr, s);
        launch_norm_raw(r, len, n1, w, s);
        hipLaunchKernelGGL(adapt_decide_kernel, dim3(1), dim3(1), 0, s, n0, n1, skip, passes, enable);
        GKL_LAUNCH_CHECK("adapt_decide_kernel");
        proj(skip);
        launch_update(Q, ldq, len, ncols, r, h1, enable, skip, s);
    } else {
        proj(nullptr);
        launch_update(Q, ldq, len, ncols, r, h1, enable, nullptr, s);
        proj(nullptr);
        // the second update also leaves the partial sums of ||r||^2 in w.npart
        launch_update(Q, ldq, len, ncols, r, h1, enable, nullptr, s, w.npart, passes);
    }
}

// ---------------------------------------------------------------------------
// Normalisation with breakdown test
// ---------------------------------------------------------------------------
__global__ void scale_kernel(const double* __restrict__ r, int64_t len, double* __restrict__ out,
                             const double* __restrict__ nrm)
{
    const double a = *nrm;
    if (a == 0.0) return;
    const double inv = 1.0 / a;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = r[i] * inv;
}

void launch_norm(const double* r, int64_t len, double* out, OrthoWork& w, hipStream_t s)
{
    launch_norm_raw(r, len, out, w, s);
}

// Normalisation right after a non-adaptive CGS2 whose second update left the
// partial sums of ||r||^2 in npart (one per 256 rows).  Every block adds the
// partials in the same order, applies the breakdown test of norm_kernel and
// scales its rows; block 0 records the results.  When *enable == 0 the CGS2 was
// skipped and *nrm_out already holds ||r|| (computed before it).  Blocks may see
// *norm_est before or after block 0 updates it: est = max(est, nrm) is the same
// either way, and so is *nrm_out (unchanged, or 0 exactly when all blocks found
// a breakdown).
__global__ void __launch_bounds__(kOT)
normalize_fused_kernel(double* __restrict__ r, int64_t len, double* nrm_out, double* norm_est,
                       double root_maxdim, int* __restrict__ flag, int* __restrict__ first_breakdown,
                       int step, const double* __restrict__ npart, int nparts,
                       const int* __restrict__ enable)
{
    __shared__ double sh[16];
    double nrm;
    if (enable && *enable == 0) {
        nrm = *nrm_out;
    } else {
        double t = 0.0;
        for (int b = threadIdx.x; b < nparts; b += kOT) t += npart[b];
        nrm = sqrt(block_sum(t, sh));
    }
    double est = *norm_est;
    if (nrm > est) est = nrm;
    const bool bd = nrm <= 2.220446049250313e-16 * est * root_maxdim;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *nrm_out = bd ? 0.0 : nrm;
        *flag = bd ? 1 : 0;
        if (bd && first_breakdown && *first_breakdown < 0) *first_breakdown = step;
        *norm_est = est;
    }
    if (bd) return;
    const double inv = 1.0 / nrm;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        r[i] = r[i] * inv;
}

void launch_normalize_after_cgs2(double* r, int64_t len, double* nrm_out, double* norm_est,
                                 double root_maxdim, int* flag, const int* enable, OrthoWork& w,
                                 hipStream_t s, int* first_breakdown, int step)
{
    unsigned int nb = ceil_div(len, 4 * kOT);
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(normalize_fused_kernel, dim3(nb), dim3(kOT), 0, s, r, len, nrm_out, norm_est,
                       root_maxdim, flag, first_breakdown, step, w.npart, (int)ceil_div(len, kOT),
                       enable);
    GKL_LAUNCH_CHECK("normalize_fused_kernel");
}

void launch_normalize(double* r, int64_t len, double* out, double* nrm_out, double* norm_est,
                      double root_maxdim, int* flag, OrthoWork& w, hipStream_t s,
                      int* first_breakdown, int step)
{
    hipLaunchKernelGGL(norm_kernel, dim3(ceil_div(len, kNRows)), dim3(kOT), 0, s, r, len, nrm_out,
                       norm_est, root_maxdim, flag, first_breakdown, step, 1, w.partial,
                       w.counters + 1);
    GKL_LAUNCH_CHECK("norm_kernel");
    unsigned int nb = ceil_div(len, 256);
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(scale_kernel, dim3(nb), dim3(256), 0, s, r, len, out, nrm_out);
    GKL_LAUNCH_CHECK("scale_kernel");
}

// ---------------------------------------------------------------------------
// y -= Q c
// ---------------------------------------------------------------------------
__global__ void gemv_n_sub_kernel(const double* __restrict__ Q, int64_t ldq, int64_t len, int ncols,
                                  const double* __restrict__ c, double* __restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        double a = y[i];
        for (int k = 0; k < ncols; ++k) a = fma(-Q[(int64_t)k * ldq + i], c[k], a);
        y[i] = a;
    }
}

void launch_gemv_n_sub(const double* Q, int64_t ldq, int64_t len, int ncols, const double* c,
                       double* y, hipStream_t s)
{
    if (ncols <= 0) return;
    unsigned int nb = ceil_div(len, 256);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(gemv_n_sub_kernel, dim3(nb), dim3(256), 0, s, Q, ldq, len, ncols, c, y);
    GKL_LAUNCH_CHECK("gemv_n_sub_kernel");
}

// ---------------------------------------------------------------------------
// C = Q S, tall-skinny: len x nin times nin x nout; 16 output columns per block row
// ---------------------------------------------------------------------------
constexpr int kGT = 16;

__global__ void __launch_bounds__(256)
gemm_tall_kernel(const double* __restrict__ Q, int64_t ldq, int64_t len, int nin,
                 const double* __restrict__ S, int lds, int nout, double* __restrict__ C,
                 int64_t ldc, int use_lds)
{
    extern __shared__ double ss[];   // nin x kGT tile of S when it fits
    const int o0 = blockIdx.y * kGT;
    const int no = nout - o0 < kGT ? nout - o0 : kGT;
    if (use_lds) {
        for (int t = threadIdx.x; t < nin * kGT; t += blockDim.x) {
            const int c = t / kGT, o = t % kGT;
            ss[t] = o < no ? S[(int64_t)(o0 + o) * lds + c] : 0.0;
        }
        __syncthreads();
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        double acc[kGT];
#pragma unroll
        for (int o = 0; o < kGT; ++o) acc[o] = 0.0;
        for (int c = 0; c < nin; ++c) {
            const double q = Q[(int64_t)c * ldq + i];
            if (use_lds) {
#pragma unroll
                for (int o = 0; o < kGT; ++o) acc[o] = fma(q, ss[c * kGT + o], acc[o]);
            } else {
#pragma unroll
                for (int o = 0; o < kGT; ++o)
                    if (o < no) acc[o] = fma(q, S[(int64_t)(o0 + o) * lds + c], acc[o]);
            }
        }
#pragma unroll
        for (int o = 0; o < kGT; ++o)
            if (o < no) C[(int64_t)(o0 + o) * ldc + i] = acc[o];
    }
}

void launch_gemm_tall(const double* Q, int64_t ldq, int64_t len, int ncols_in, const double* S,
                      int lds, int ncols_out, double* C, int64_t ldc, hipStream_t s)
{
    if (ncols_out <= 0 || len <= 0) return;
    unsigned int nb = ceil_div(len, 256);
    if (nb > 2048) nb = 2048;
    dim3 grid(nb, ceil_div(ncols_out, kGT));
    const int use_lds = (size_t)ncols_in * kGT * sizeof(double) <= 32768 ? 1 : 0;
    const size_t shmem = use_lds ? sizeof(double) * (size_t)(ncols_in > 0 ? ncols_in : 1) * kGT : 0;
    hipLaunchKernelGGL(gemm_tall_kernel, grid, dim3(256), shmem, s, Q, ldq, len, ncols_in, S,
                       lds, ncols_out, C, ldc, use_lds);
    GKL_LAUNCH_CHECK("gemm_tall_kernel");
}

// ---------------------------------------------------------------------------
// Seeded Gaussian vector: SplitMix64 output function on (seed, stream, index),
// Box-Muller on two 53-bit uniforms.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void gaussian_kernel(double* __restrict__ x, int64_t len, uint64_t seed, uint64_t sid)
{
    const uint64_t key = mix64(mix64(seed) ^ (sid * 0xD1B54A32D192ED03ull));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t a = mix64(key + 2 * (uint64_t)i);
        const uint64_t b = mix64(key + 2 * (uint64_t)i + 1);
        const double u1 = ((double)(a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
        x[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}

void launch_gaussian(double* x, int64_t len, uint64_t seed, uint64_t stream_id, hipStream_t s)
{
    unsigned int nb = ceil_div(len, 256);
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(gaussian_kernel, dim3(nb), dim3(256), 0, s, x, len, seed, stream_id);
    GKL_LAUNCH_CHECK("gaussian_kernel");
}

// ---------------------------------------------------------------------------
// Sign rule: largest |V(:, c)| entry positive, lowest index on ties.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
sign_fix_kernel(double* __restrict__ U, int64_t ldu, int64_t n, double* __restrict__ V,
                int64_t ldv, int64_t p)
{
    __shared__ double bv[4];
    __shared__ int64_t bi[4];
    __shared__ int flip;
    const int c = blockIdx.x;
    double* v = V + (int64_t)c * ldv;
    double best = -1.0;
    int64_t bidx = INT64_MAX;
    for (int64_t i = threadIdx.x; i < p; i += blockDim.x) {
        const double a = fabs(v[i]);
        if (a > best) { best = a; bidx = i; }      // strided ascending: first max kept
    }
    // wave argmax (larger value, then lower index)
    for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int64_t oi = __shfl_xor(bidx, off, 64);
        if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { bv[wid] = best; bi[wid] = bidx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = bv[0];
        int64_t ix = bi[0];
        for (int w = 1; w < (int)(blockDim.x / 64); ++w)
            if (bv[w] > b || (bv[w] == b && bi[w] < ix)) { b = bv[w]; ix = bi[w]; }
        flip = (ix < p && v[ix] < 0.0) ? 1 : 0;
    }
    __syncthreads();
    if (!flip) return;
    for (int64_t i = threadIdx.x; i < p; i += blockDim.x) v[i] = -v[i];
    double* u = U + (int64_t)c * ldu;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) u[i] = -u[i];
}

void launch_sign_fix(double* U, int64_t ldu, int64_t n, double* V, int64_t ldv, int64_t p, int k,
                     hipStream_t s)
{
    if (k <= 0) return;
    hipLaunchKernelGGL(sign_fix_kernel, dim3(k), dim3(256), 0, s, U, ldu, n, V, ldv, p);
    GKL_LAUNCH_CHECK("sign_fix_kernel");
}

}  // namespace gkl
