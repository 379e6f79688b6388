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
// contiguous rows; reductions over rows are two-stage with a fixed order (block
// partials, then the last block to arrive sums them), hence deterministic.
#include <math.h>

#include "engine.h"

namespace gkl {

namespace {
constexpr int kOT = 256;     // threads per block
constexpr int kORows = 2;    // rows per thread
constexpr int kORowsPerBlock = kOT * kORows;
}  // namespace

size_t ortho_partial_elems(int64_t len, int maxcols)
{
    return (size_t)ceil_div(len, kORowsPerBlock) * (size_t)(maxcols + 2);
}

// One pass over the rows of r:
//   if hin:        r <- r - Q hin      (hin: ncols, skipped when *skip != 0)
//   if hout:       partials of Q^T r   -> hout (ncols) by the last block
//   if nrm2_out:   partial of ||r||^2  -> *nrm2_out by the last block
// After the reduction the last block may apply the adaptive test: when
// adapt_ref (||r_before||^2) is given and ||r||^2 >= adapt_ref / 2 it sets
// *skip_next = 1 (no second pass), else 0 and counts a pass.
__global__ void __launch_bounds__(kOT)
ortho_pass_kernel(const double* __restrict__ Q, int64_t ldq, int64_t len, int ncols,
                  double* __restrict__ r, const int* __restrict__ enable,
                  const double* __restrict__ hin, const int* __restrict__ skip,
                  double* __restrict__ hout, double* __restrict__ nrm2_out,
                  const double* __restrict__ adapt_ref, int* __restrict__ skip_next,
                  int* __restrict__ passes, double* __restrict__ partial,
                  unsigned int* __restrict__ counter)
{
    if (enable && *enable == 0) return;
    extern __shared__ double sh[];          // ncols (hin) + 4 * (ncols + 1) wave partials
    double* hs = sh;
    double* wp = sh + ncols;
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * kORowsPerBlock + threadIdx.x;
    double rv[kORows];
#pragma unroll
    for (int t = 0; t < kORows; ++t) {
        const int64_t row = row0 + t * kOT;
        rv[t] = row < len ? r[row] : 0.0;
    }
    const bool do_update = hin != nullptr && !(skip && *skip);
    if (do_update) {
        for (int c = threadIdx.x; c < ncols; c += kOT) hs[c] = hin[c];
        __syncthreads();
        for (int c = 0; c < ncols; ++c) {
            const double hc = hs[c];
            const double* qc = Q + (int64_t)c * ldq;
#pragma unroll
            for (int t = 0; t < kORows; ++t) {
                const int64_t row = row0 + t * kOT;
                if (row < len) rv[t] = fma(-qc[row], hc, rv[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < kORows; ++t) {
            const int64_t row = row0 + t * kOT;
            if (row < len) r[row] = rv[t];
        }
    }
    const int nout = (hout ? ncols : 0) + (nrm2_out ? 1 : 0);
    if (nout == 0) return;
    if (hout) {
        for (int c = 0; c < ncols; ++c) {
            const double* qc = Q + (int64_t)c * ldq;
            double a = 0.0;
#pragma unroll
            for (int t = 0; t < kORows; ++t) {
                const int64_t row = row0 + t * kOT;
                if (row < len) a = fma(qc[row], rv[t], a);
            }
            a = wave_sum(a);
            if (lane == 0) wp[wid * (ncols + 1) + c] = a;
        }
    }
    if (nrm2_out) {
        double a = 0.0;
#pragma unroll
        for (int t = 0; t < kORows; ++t) a = fma(rv[t], rv[t], a);
        a = wave_sum(a);
        if (lane == 0) wp[wid * (ncols + 1) + ncols] = a;
    }
    __syncthreads();
    const int stride = ncols + 1;
    for (int c = threadIdx.x; c < stride; c += kOT) {
        if (c < ncols && !hout) continue;
        if (c == ncols && !nrm2_out) continue;
        double a = 0.0;
        for (int w = 0; w < kOT / 64; ++w) a += wp[w * stride + c];
        partial[(int64_t)blockIdx.x * stride + c] = a;
    }
    if (!last_block_arrived(counter, gridDim.x)) return;
    for (int c = threadIdx.x; c < stride; c += kOT) {
        if (c < ncols && !hout) continue;
        if (c == ncols && !nrm2_out) continue;
        double a = 0.0;
        for (unsigned int b = 0; b < gridDim.x; ++b) a += partial[(int64_t)b * stride + c];
        if (c < ncols) hout[c] = a;
        else *nrm2_out = a;
    }
    if (threadIdx.x == 0 && skip_next) {
        // nrm2_out holds ||r after first pass||^2 here; adapt_ref the norm before it
        __threadfence_block();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (skip_next && adapt_ref && nrm2_out) {
            const double after = *nrm2_out;
            const int sk = (after >= 0.5 * (*adapt_ref)) ? 1 : 0;
            *skip_next = sk;
            if (passes) *passes += sk ? 1 : 2;
        } else if (passes && hin == nullptr && hout) {
            // non-adaptive: counted once per CGS2 call by the first pass
            *passes += 2;
        }
    }
}

static void ortho_pass(const double* Q, int64_t ldq, int64_t len, int ncols, double* r,
                       const int* enable, const double* hin, const int* skip, double* hout,
                       double* nrm2_out, const double* adapt_ref, int* skip_next, int* passes,
                       OrthoWork& w, hipStream_t s)
{
    const unsigned int nb = ceil_div(len, kORowsPerBlock);
    const size_t shmem = sizeof(double) * ((size_t)ncols + 4 * ((size_t)ncols + 1));
    hipLaunchKernelGGL(ortho_pass_kernel, dim3(nb), dim3(kOT), shmem, s, Q, ldq, len, ncols, r,
                       enable, hin, skip, hout, nrm2_out, adapt_ref, skip_next, passes, w.partial,
                       w.counters);
    GKL_LAUNCH_CHECK("ortho_pass_kernel");
}

void launch_cgs2(const double* Q, int64_t ldq, int64_t len, int ncols, double* r,
                 const int* enable, int adaptive, int* passes, OrthoWork& w, hipStream_t s)
{
    if (ncols <= 0) return;
    double* h1 = w.h;
    double* h2 = w.h + (ncols + 1);
    double* n0 = w.h + 2 * (ncols + 1);
    double* n1 = n0 + 1;
    int* skip = reinterpret_cast<int*>(n0 + 2);
    if (adaptive) {
        // pass 1: h1 = Q^T r, ||r||^2
        ortho_pass(Q, ldq, len, ncols, r, enable, nullptr, nullptr, h1, n0, nullptr, nullptr,
                   nullptr, w, s);
        // pass 2: r -= Q h1; h2 = Q^T r; ||r||^2; decide whether a second update is needed
        ortho_pass(Q, ldq, len, ncols, r, enable, h1, nullptr, h2, n1, n0, skip, passes, w, s);
        // pass 3: r -= Q h2 unless skipped
        ortho_pass(Q, ldq, len, ncols, r, enable, h2, skip, nullptr, nullptr, nullptr, nullptr,
                   nullptr, w, s);
    } else {
        ortho_pass(Q, ldq, len, ncols, r, enable, nullptr, nullptr, h1, nullptr, nullptr,
                   nullptr, passes, w, s);
        ortho_pass(Q, ldq, len, ncols, r, enable, h1, nullptr, h2, nullptr, nullptr, nullptr,
                   nullptr, w, s);
        ortho_pass(Q, ldq, len, ncols, r, enable, h2, nullptr, nullptr, nullptr, nullptr,
                   nullptr, nullptr, w, s);
    }
}

// ---------------------------------------------------------------------------
// Normalisation with breakdown test
// ---------------------------------------------------------------------------
__global__ void normalize_decide_kernel(const double* __restrict__ nrm2, double* __restrict__ nrm_out,
                                        double* __restrict__ norm_est, double root_maxdim,
                                        int* __restrict__ flag)
{
    const double nrm = sqrt(*nrm2);
    double est = *norm_est;
    if (nrm > est) est = nrm;
    const double thresh = 2.220446049250313e-16 * est * root_maxdim;
    if (nrm <= thresh) {
        *nrm_out = 0.0;
        *flag = 1;
    } else {
        *nrm_out = nrm;
        *flag = 0;
    }
    *norm_est = est;
}

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

__global__ void sqrt_kernel(const double* __restrict__ a, double* __restrict__ out)
{
    *out = sqrt(*a);
}

void launch_norm(const double* r, int64_t len, double* out, OrthoWork& w, hipStream_t s)
{
    double* n2 = w.h + 1;
    ortho_pass(nullptr, 0, len, 0, const_cast<double*>(r), nullptr, nullptr, nullptr, nullptr, n2,
               nullptr, nullptr, nullptr, w, s);
    hipLaunchKernelGGL(sqrt_kernel, dim3(1), dim3(1), 0, s, n2, out);
    GKL_LAUNCH_CHECK("sqrt_kernel");
}

void launch_normalize(double* r, int64_t len, double* out, double* nrm_out, double* norm_est,
                      double root_maxdim, int* flag, OrthoWork& w, hipStream_t s)
{
    double* n2 = w.h + 0;
    ortho_pass(nullptr, 0, len, 0, r, nullptr, nullptr, nullptr, nullptr, n2, nullptr, nullptr,
               nullptr, w, s);
    hipLaunchKernelGGL(normalize_decide_kernel, dim3(1), dim3(1), 0, s, n2, nrm_out, norm_est,
                       root_maxdim, flag);
    GKL_LAUNCH_CHECK("normalize_decide_kernel");
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
