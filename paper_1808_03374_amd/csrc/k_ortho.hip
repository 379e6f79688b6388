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
// contiguous rows.  The two-pass CGS2 takes three launches: projection partials;
// update by the first projection fused with the partials of the second; update
// by the second with the norm partials.  Each launch sums the previous one's
// partials itself, in a fixed order, so no reduction launches sit between them.
// Norms are two-stage reductions with a fixed order.  All results are
// deterministic.
#include <math.h>

#include <algorithm>

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

// ---------------------------------------------------------------------------
// Two-pass CGS2 of one vector in three launches
// ---------------------------------------------------------------------------
// Each wave owns one tile of 64 consecutive rows (lane = row) and each
// workgroup kCT / 64 tiles, so every pass touches the same rows from the same
// lane and r is updated in place without cross-workgroup hazards.  A lane loads
// its row of up to 64 basis columns at once (one coalesced 512-byte access per
// column and wave); for ncols <= 64 those values stay in registers, so the
// update and the next projection share one read of Q.  The column sums over a
// wave are formed by a transpose-sum (lane l ends with column l), then the
// waves of a workgroup are added in order: part[b * cstride + c].
namespace {
constexpr int kCT = 512;          // threads per workgroup
constexpr int kCW = kCT / 64;     // waves (tiles) per workgroup
constexpr int kCChunk = 64;       // columns per chunk (one per lane)
}  // namespace

struct CgsPlan {
    int nb;        // workgroups
    int cstride;   // partial row stride (ncols rounded up to kCChunk)
};

static CgsPlan cgs_plan(int64_t len, int ncols)
{
    CgsPlan c;
    c.nb = (int)ceil_div(len, kCT);
    c.cstride = (int)ceil_div(ncols, kCChunk) * kCChunk;
    return c;
}

size_t cgs_partial_elems(int64_t len, int maxcols)
{
    const CgsPlan c = cgs_plan(len, maxcols);
    return 2 * (size_t)c.nb * (size_t)c.cstride;
}

int cgs_norm_partials(int64_t len)
{
    return cgs_plan(len, 1).nb;
}

// Lane exchanges for the transpose-sum.  swap32 / swap16: the two halves
// (rows of 16) of a pair of registers change places between lanes l and l ^ 32
// (l ^ 16).  xor8 .. xor1: the value of lane l ^ d within a row of 16 (DPP:
// rotate by 8; half-row mirror after a quad reversal; quad permutes).
__device__ __forceinline__ void swap_halves32(double& a, double& b)
{
    const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)y, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(x >> 32), (unsigned)(y >> 32),
                                                     false, false);
    a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
    b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

__device__ __forceinline__ void swap_halves16(double& a, double& b)
{
    const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)y, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(x >> 32), (unsigned)(y >> 32),
                                                     false, false);
    a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
    b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

template <int kCtrl>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, kCtrl, 0xF, 0xF, false);
}

template <int kD>
__device__ __forceinline__ double lane_xor(double v)
{
    const long long x = __double_as_longlong(v);
    int lo = (int)(x & 0xffffffff), hi = (int)(x >> 32);
    if (kD == 8) { lo = dpp_i<0x128>(lo); hi = dpp_i<0x128>(hi); }            // row_ror:8
    if (kD == 4) {                                                             // quad reverse,
        lo = dpp_i<0x141>(dpp_i<0x1B>(lo)); hi = dpp_i<0x141>(dpp_i<0x1B>(hi)); // half mirror
    }
    if (kD == 2) { lo = dpp_i<0x4E>(lo); hi = dpp_i<0x4E>(hi); }              // [2,3,0,1]
    if (kD == 1) { lo = dpp_i<0xB1>(lo); hi = dpp_i<0xB1>(hi); }              // [1,0,3,2]
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Round of distance kD <= 8 on v[0..2 kD): lane keeps column i + kD when its
// bit kD is set, else column i, adding the partner's copy of the same column.
template <int kD>
__device__ __forceinline__ void xor_round(double (&v)[kCChunk], bool hi)
{
#pragma unroll
    for (int i = 0; i < kD; ++i) {
        const double lo_sum = v[i] + lane_xor<kD>(v[i]);
        const double hi_sum = v[i + kD] + lane_xor<kD>(v[i + kD]);
        v[i] = hi ? hi_sum : lo_sum;
    }
}

// v[0..64) held by every lane of a wave; returns to lane l the sum over the
// wave of v[l].  Six exchange rounds of distance d = 32 .. 1: each lane keeps
// the half of its live values whose column has bit d equal to its own lane
// bit d and adds the partner's (lane l ^ d) copy of that half.  The rounds of
// distance 32 and 16 swap register halves between lanes, so every lane adds
// the pair it ends up with; the others exchange both halves and keep one sum.
// Additions are commutative pairs in a fixed pattern, so the result is
// deterministic.
__device__ __forceinline__ double wave_transpose_sum(double (&v)[kCChunk], int lane)
{
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        swap_halves32(v[i], v[i + 32]);
        v[i] = v[i] + v[i + 32];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        swap_halves16(v[i], v[i + 16]);
        v[i] = v[i] + v[i + 16];
    }
    xor_round<8>(v, (lane & 8) != 0);
    xor_round<4>(v, (lane & 4) != 0);
    xor_round<2>(v, (lane & 2) != 0);
    xor_round<1>(v, (lane & 1) != 0);
    return v[0];
}

// Row `rowc` of columns [c0, c0 + 64) into q; columns at or past ncols read
// column ncols - 1 again (in bounds).  Their values only reach partials past
// ncols, which are never read, and updates through coefficients that are zero
// there.  The loads are unconditional so they are all in flight together.
__device__ __forceinline__ void load_row_chunk(const double* __restrict__ Q, int64_t ldq,
                                               int64_t rowc, int c0, int ncols,
                                               double (&q)[kCChunk])
{
    const double* qp = Q + (int64_t)c0 * ldq + rowc;
#pragma unroll
    for (int k = 0; k < kCChunk; ++k) {
        q[k] = *qp;
        if (k + 1 < kCChunk) qp += (c0 + k + 1 < ncols) ? ldq : 0;
    }
}

// Adds the wave's column sums sw (lane l: column c0 + l) of every wave in order
// and stores them at out[c0 + l]; red holds kCW x 64 doubles.
__device__ __forceinline__ void block_columns(double sw, double* red, double* __restrict__ out,
                                              int c0)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    __syncthreads();
    red[wave * 64 + lane] = sw;
    __syncthreads();
    if (t < 64) {
        double h = red[t];
#pragma unroll
        for (int w = 1; w < kCW; ++w) h += red[w * 64 + t];
        out[c0 + t] = h;
    }
}

// kMode 0: partials of Q^T r.
// kMode 1: h = sum of the pass-1 partials; r -= Q h; partials of Q^T r.
// kMode 2: h = sum of the pass-2 partials; r -= Q h; npart[b] = sum of the
//          squares of the workgroup's updated rows; block 0 adds 2 to *passes.
// With *enable == 0 every workgroup returns at once (the same for all).
template <int kMode>
__global__ void __launch_bounds__(kCT)
cgs_pass_kernel(const double* __restrict__ Q, int64_t ldq, int64_t len, int ncols,
                double* __restrict__ r, const double* __restrict__ pin,
                double* __restrict__ pout, int nb, int cstride, const int* __restrict__ enable,
                int* __restrict__ passes)
{
    if (enable && *enable == 0) return;
    extern __shared__ double hs[];             // cstride coefficients (kMode > 0)
    __shared__ double red[kCW * 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t row = (int64_t)blockIdx.x * kCT + t;
    const bool live = row < len;
    const int64_t rowc = live ? row : len - 1;

    if (kMode > 0) {   // coefficients, zero past ncols
        for (int c0 = 0; c0 < ncols; c0 += kCChunk) {
            const int c = c0 + lane;
            double sacc = 0.0;
            if (c < ncols) {
#pragma unroll 4
                for (int b = wave; b < nb; b += kCW) sacc += pin[(int64_t)b * cstride + c];
            }
            __syncthreads();
            red[wave * 64 + lane] = sacc;
            __syncthreads();
            if (t < 64) {
                double h = red[t];
#pragma unroll
                for (int w = 1; w < kCW; ++w) h += red[w * 64 + t];
                hs[c0 + t] = c < ncols ? h : 0.0;
            }
        }
        __syncthreads();
    }

    double x = live ? r[row] : 0.0;
    double q[kCChunk];
    if (ncols <= kCChunk) {
        load_row_chunk(Q, ldq, rowc, 0, ncols, q);
        if (kMode > 0) {
#pragma unroll
            for (int k = 0; k < kCChunk; ++k) x = fma(-q[k], hs[k], x);
            if (live) r[row] = x;
            x = live ? x : 0.0;     // lanes past len read row len - 1: no contribution
        }
        if (kMode == 2) {
            const double ss = block_sum(x * x, red);
            if (t == 0) pout[blockIdx.x] = ss;
            if (passes && blockIdx.x == 0 && t == 0) *passes += 2;
            return;
        }
#pragma unroll
        for (int k = 0; k < kCChunk; ++k) q[k] *= x;
        block_columns(wave_transpose_sum(q, lane), red, pout + (int64_t)blockIdx.x * cstride, 0);
        return;
    }
    // more than 64 columns: update over all chunks first, then the projection
    // reads the chunks again
    if (kMode > 0) {
        for (int c0 = 0; c0 < ncols; c0 += kCChunk) {
            load_row_chunk(Q, ldq, rowc, c0, ncols, q);
#pragma unroll
            for (int k = 0; k < kCChunk; ++k) x = fma(-q[k], hs[c0 + k], x);
        }
        if (live) r[row] = x;
        x = live ? x : 0.0;
    }
    if (kMode == 2) {
        const double ss = block_sum(x * x, red);
        if (t == 0) pout[blockIdx.x] = ss;
        if (passes && blockIdx.x == 0 && t == 0) *passes += 2;
        return;
    }
    for (int c0 = 0; c0 < ncols; c0 += kCChunk) {
        load_row_chunk(Q, ldq, rowc, c0, ncols, q);
#pragma unroll
        for (int k = 0; k < kCChunk; ++k) q[k] *= x;
        block_columns(wave_transpose_sum(q, lane), red, pout + (int64_t)blockIdx.x * cstride, c0);
    }
}

// The same three passes for a block of kB <= 4 vectors (Y, column-major, ld
// ldy) against Q, without the norm tail: the blocked GKL's block Gram-Schmidt
// (the block QR that follows orthonormalises the block itself).  Each
// workgroup reads its rows of Q once per pass for all kB vectors, so CGS2
// costs three passes over Q; partials of vector v at pout + (wg kB + v) cstride.
// Between passes a separate kernel adds the partials once (with a basis of up
// to 130 columns and ~1,000 workgroups, every workgroup adding them itself
// read gigabytes from L2); hin holds the kB x cstride coefficients.
template <int kMode, int kB>
__global__ void __launch_bounds__(kCT)
cgs_block_pass_kernel(const double* __restrict__ Q, int64_t ldq, int64_t len, int ncols,
                      double* __restrict__ Y, int64_t ldy, const double* __restrict__ hin,
                      double* __restrict__ pout, int cstride)
{
    extern __shared__ double hs[];             // kB x cstride coefficients (kMode > 0)
    __shared__ double red[kCW * 64];
    const int t = threadIdx.x, lane = t & 63;
    const int64_t row = (int64_t)blockIdx.x * kCT + t;
    const bool live = row < len;
    const int64_t rowc = live ? row : len - 1;

    if (kMode > 0) {
        for (int e = t; e < kB * cstride; e += kCT) hs[e] = hin[e];
        __syncthreads();
    }

    // Columns are taken kW at a time, kW = 64 / kP with kP >= kB slots: the
    // products of the kB vectors with one chunk fill one 64-entry array (slot v
    // at kW v .. kW v + kW - 1), so one wave transpose-sum serves them all and
    // every chunk is read once per pass.
    constexpr int kP = kB == 1 ? 1 : kB == 2 ? 2 : 4;
    constexpr int kW = kCChunk / kP;
    double x[kB];
#pragma unroll
    for (int v = 0; v < kB; ++v) x[v] = live ? Y[(int64_t)v * ldy + row] : 0.0;
    double q[kW];
    auto load_chunk = [&](int c0) {
        const double* qp = Q + (int64_t)c0 * ldq + rowc;
#pragma unroll
        for (int k = 0; k < kW; ++k) {   // columns past ncols read column ncols - 1 again
            q[k] = *qp;
            if (k + 1 < kW) qp += (c0 + k + 1 < ncols) ? ldq : 0;
        }
    };
    if (kMode > 0) {
        for (int c0 = 0; c0 < ncols; c0 += kW) {
            load_chunk(c0);
#pragma unroll
            for (int v = 0; v < kB; ++v)
#pragma unroll
                for (int k = 0; k < kW; ++k) x[v] = fma(-q[k], hs[v * cstride + c0 + k], x[v]);
        }
#pragma unroll
        for (int v = 0; v < kB; ++v) {
            if (live) Y[(int64_t)v * ldy + row] = x[v];
            x[v] = live ? x[v] : 0.0;   // lanes past len read row len - 1: no contribution
        }
    }
    if (kMode == 2) return;
    for (int c0 = 0; c0 < ncols; c0 += kW) {
        // with one chunk the rows loaded for the update are still in q
        if (kMode == 0 || ncols > kW) load_chunk(c0);
        double tmp[kCChunk];
#pragma unroll
        for (int v = 0; v < kP; ++v)
#pragma unroll
            for (int k = 0; k < kW; ++k) tmp[v * kW + k] = v < kB ? q[k] * x[v < kB ? v : 0] : 0.0;
        const double sw = wave_transpose_sum(tmp, lane);   // lane l: slot l / kW, column c0 + l % kW
        __syncthreads();
        red[(t >> 6) * 64 + lane] = sw;
        __syncthreads();
        if (t < 64) {
            double h = red[t];
#pragma unroll
            for (int w = 1; w < kCW; ++w) h += red[w * 64 + t];
            const int v = t / kW;
            if (v < kB) pout[((int64_t)blockIdx.x * kB + v) * cstride + c0 + t % kW] = h;
        }
    }
}

// h[v cstride + c] = sum over the nb workgroup partials of column c of vector
// v (zero for ncols <= c < cstride): one wave per coefficient, lane l adding
// workgroups l, l + 64, ... in order, then a fixed butterfly.
__global__ void __launch_bounds__(256)
cgs_block_sum_kernel(const double* __restrict__ pin, int nb, int kb, int ncols, int cstride,
                     double* __restrict__ h)
{
    const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (o >= kb * cstride) return;              // the whole wave
    const int v = o / cstride, c = o - v * cstride;
    double sum = 0.0;
    if (c < ncols)
        for (int b = lane; b < nb; b += 64) sum += pin[((int64_t)b * kb + v) * cstride + c];
    sum = wave_sum(sum);
    if (lane == 0) h[o] = sum;
}

template <int kB>
static void block_cgs2_run(const double* Q, int64_t ldq, int64_t len, int ncols, double* Y,
                           int64_t ldy, double* partial, size_t partial_elems, hipStream_t s)
{
    const CgsPlan c = cgs_plan(len, ncols);
    const size_t pe = (size_t)c.nb * kB * c.cstride;
    const size_t he = (size_t)kB * c.cstride;
    if (2 * pe + 2 * he > partial_elems)
        fail(GKL_ERR_INTERNAL, "block CGS2 plan exceeds its partial buffer");
    double* p1 = partial;
    double* p2 = partial + pe;
    double* h1 = partial + 2 * pe;
    double* h2 = h1 + he;
    const size_t hb = sizeof(double) * he;
    const dim3 gsum((unsigned int)ceil_div((int64_t)he, 4));
    hipLaunchKernelGGL((cgs_block_pass_kernel<0, kB>), dim3(c.nb), dim3(kCT), 0, s, Q, ldq, len,
                       ncols, Y, ldy, nullptr, p1, c.cstride);
    GKL_LAUNCH_CHECK("cgs_block_pass_kernel<0>");
    hipLaunchKernelGGL(cgs_block_sum_kernel, gsum, dim3(256), 0, s, p1, c.nb, kB, ncols, c.cstride, h1);
    GKL_LAUNCH_CHECK("cgs_block_sum_kernel");
    hipLaunchKernelGGL((cgs_block_pass_kernel<1, kB>), dim3(c.nb), dim3(kCT), hb, s, Q, ldq, len,
                       ncols, Y, ldy, h1, p2, c.cstride);
    GKL_LAUNCH_CHECK("cgs_block_pass_kernel<1>");
    hipLaunchKernelGGL(cgs_block_sum_kernel, gsum, dim3(256), 0, s, p2, c.nb, kB, ncols, c.cstride, h2);
    GKL_LAUNCH_CHECK("cgs_block_sum_kernel");
    hipLaunchKernelGGL((cgs_block_pass_kernel<2, kB>), dim3(c.nb), dim3(kCT), hb, s, Q, ldq, len,
                       ncols, Y, ldy, h2, nullptr, c.cstride);
    GKL_LAUNCH_CHECK("cgs_block_pass_kernel<2>");
}

size_t block_cgs2_partial_elems(int64_t len, int maxcols, int b)
{
    const CgsPlan c = cgs_plan(len, maxcols);
    return 2 * (size_t)c.nb * (size_t)b * (size_t)c.cstride + 2 * (size_t)b * (size_t)c.cstride;
}

void launch_block_cgs2(const double* Q, int64_t ldq, int64_t len, int ncols, double* Y, int64_t ldy,
                       int b, double* partial, size_t partial_elems, hipStream_t s)
{
    if (ncols <= 0) return;
    switch (b) {
    case 1: block_cgs2_run<1>(Q, ldq, len, ncols, Y, ldy, partial, partial_elems, s); break;
    case 2: block_cgs2_run<2>(Q, ldq, len, ncols, Y, ldy, partial, partial_elems, s); break;
    case 3: block_cgs2_run<3>(Q, ldq, len, ncols, Y, ldy, partial, partial_elems, s); break;
    case 4: block_cgs2_run<4>(Q, ldq, len, ncols, Y, ldy, partial, partial_elems, s); break;
    default: fail(GKL_ERR_INTERNAL, "launch_block_cgs2 takes blocks of 1 to 4 vectors");
    }
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
        // the last pass also leaves the partial sums of ||r||^2 in w.npart
        const CgsPlan c = cgs_plan(len, ncols);
        if (2 * (size_t)c.nb * (size_t)c.cstride > w.cgs_partial_elems)
            fail(GKL_ERR_INTERNAL, "CGS2 plan exceeds its partial buffer");
        double* p1 = w.cgs_partial;
        double* p2 = w.cgs_partial + (size_t)c.nb * c.cstride;
        const size_t hb = sizeof(double) * (size_t)c.cstride;
        hipLaunchKernelGGL(cgs_pass_kernel<0>, dim3(c.nb), dim3(kCT), 0, s, Q, ldq, len, ncols, r,
                           nullptr, p1, c.nb, c.cstride, enable, nullptr);
        GKL_LAUNCH_CHECK("cgs_pass_kernel<0>");
        hipLaunchKernelGGL(cgs_pass_kernel<1>, dim3(c.nb), dim3(kCT), hb, s, Q, ldq, len, ncols, r,
                           p1, p2, c.nb, c.cstride, enable, nullptr);
        GKL_LAUNCH_CHECK("cgs_pass_kernel<1>");
        hipLaunchKernelGGL(cgs_pass_kernel<2>, dim3(c.nb), dim3(kCT), hb, s, Q, ldq, len, ncols, r,
                           p2, w.npart, c.nb, c.cstride, enable, passes);
        GKL_LAUNCH_CHECK("cgs_pass_kernel<2>");
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

// Normalisation right after a non-adaptive CGS2 whose last pass left the
// partial sums of ||r||^2 in npart (one per CGS2 workgroup).  Every block adds the
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
                       root_maxdim, flag, first_breakdown, step, w.npart, cgs_norm_partials(len),
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
// Overlap check of one-sided reorthogonalisation
// ---------------------------------------------------------------------------
// flag = 1 when max_i |h_i| > omega ||q||, h = Q(:, 0:ncols)^T q.
__global__ void __launch_bounds__(256)
overlap_flag_kernel(const double* __restrict__ h, int ncols, double omega,
                    const double* __restrict__ qnorm, int* __restrict__ flag)
{
    __shared__ double sh[4];
    double m = 0.0;
    for (int i = threadIdx.x; i < ncols; i += blockDim.x) m = fmax(m, fabs(h[i]));
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mx = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
        if (mx > omega * *qnorm) *flag = 1;
    }
}

void launch_overlap_check(const double* Q, int64_t len, int ncols, const double* q, double omega,
                          const double* qnorm, int* flag, OrthoWork& w, hipStream_t s)
{
    if (ncols <= 0) return;
    launch_gemm_tn(Q, len, q, len, len, ncols, 1, w.h, ncols, w.tn_partial, s);
    hipLaunchKernelGGL(overlap_flag_kernel, dim3(1), dim3(256), 0, s, w.h, ncols, omega, qnorm,
                       flag);
    GKL_LAUNCH_CHECK("overlap_flag_kernel");
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
