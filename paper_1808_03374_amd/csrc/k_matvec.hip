// FP64 products with the implicitly standardised genotype matrix (gfx950).
//
//   (A v)_i   = sum_j o_ij (g_ij - mu_j) s_j v_j
//   (A^T u)_j = s_j ( sum_i g_ij u_i - mu_j sum_i o_ij u_i )
//
// Section 3 of the paper: each Lanczos step applies A once and A^T once; these
// two products are where the iteration spends its time.  Genotypes stay in
// their 2-bit packed form in HBM and are decoded in registers; the dense
// standardised matrix is never formed.
//
// Both kernels stream the internal SNP-major layout (ldp bytes per column,
// ldp % 256 == 0, padding codes = 3).  A lane owns 16 individuals (one 32-bit
// word per column), so a wavefront reads 256 contiguous bytes per column.
// Partial sums over column splits (A v) or individual chunks (A^T u) are
// combined by the last block to arrive, in a fixed order (deterministic).
#include "kernels.h"

namespace gkl {

namespace {

constexpr int kThreads = 256;
constexpr int kIndPerThread = 16;
constexpr int kIndPerBlock = kThreads * kIndPerThread;   // 4096

struct MvGrid {
    unsigned int gx, gy;
    int64_t cols_per_split;
};

MvGrid matvec_grid(const Packed& P)
{
    MvGrid g;
    g.gx = ceil_div(P.ldp * 4, kIndPerBlock);
    // aim for >= 2048 blocks so the 256 CUs stay busy
    int64_t splits = (2048 + g.gx - 1) / g.gx;
    if (splits > P.p) splits = P.p;
    if (splits < 1) splits = 1;
    g.cols_per_split = (P.p + splits - 1) / splits;
    g.gy = (unsigned int)((P.p + g.cols_per_split - 1) / g.cols_per_split);
    return g;
}

constexpr int64_t kRCols = 128;   // columns per block in A^T u

}  // namespace

size_t matvec_partial_elems(const Packed& P)
{
    MvGrid g = matvec_grid(P);
    const size_t a = (size_t)g.gy * (size_t)g.gx * kIndPerBlock;       // A v partials
    const size_t nchunks = (size_t)ceil_div(P.ldp * 4, kWave * kIndPerThread);
    const size_t b = nchunks * (size_t)P.p * 2;                          // A^T u partials
    return a > b ? a : b;
}

size_t matvec_counters(const Packed& P)
{
    MvGrid g = matvec_grid(P);
    const size_t a = g.gx;
    const size_t b = ceil_div(P.p, kRCols);
    return a > b ? a : b;
}

// ---------------------------------------------------------------------------
// y = A v - beta * uprev
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
matvec_kernel(const uint32_t* __restrict__ G, int64_t n, int64_t p, int64_t ldw,
              const double* __restrict__ mean, const double* __restrict__ inv_sd,
              const double* __restrict__ v, int64_t cols_per_split, double* __restrict__ partial,
              unsigned int* __restrict__ counters, double* __restrict__ y,
              const double* __restrict__ beta, const double* __restrict__ uprev)
{
    const int64_t dw = (int64_t)blockIdx.x * kThreads + threadIdx.x;   // word within a column
    const int64_t j0 = (int64_t)blockIdx.y * cols_per_split;
    const int64_t j1 = j0 + cols_per_split < p ? j0 + cols_per_split : p;
    double acc[kIndPerThread];
#pragma unroll
    for (int k = 0; k < kIndPerThread; ++k) acc[k] = 0.0;
    if (dw < ldw) {
        const uint32_t* col = G + j0 * ldw + dw;
        for (int64_t j = j0; j < j1; ++j, col += ldw) {
            const double w = inv_sd[j] * v[j];
            const double x = mean[j] * w;
            const uint32_t word = *col;
#pragma unroll
            for (int k = 0; k < kIndPerThread; ++k) {
                const uint32_t c = (word >> (2 * k)) & 3u;
                const double t = fma((double)c, w, -x);
                acc[k] += (c == 3u) ? 0.0 : t;
            }
        }
    }
    const int64_t ind_per_split = (int64_t)gridDim.x * kIndPerBlock;
    double* my = partial + (int64_t)blockIdx.y * ind_per_split + (int64_t)blockIdx.x * kIndPerBlock;
#pragma unroll
    for (int k = 0; k < kIndPerThread; ++k) my[threadIdx.x * kIndPerThread + k] = acc[k];

    if (!last_block_arrived(&counters[blockIdx.x], gridDim.y)) return;
    const double b = beta ? *beta : 0.0;
    for (int t = threadIdx.x; t < kIndPerBlock; t += kThreads) {
        const int64_t i = (int64_t)blockIdx.x * kIndPerBlock + t;
        if (i >= n) break;
        double s = 0.0;
        for (unsigned int sp = 0; sp < gridDim.y; ++sp)
            s += partial[(int64_t)sp * ind_per_split + (int64_t)blockIdx.x * kIndPerBlock + t];
        if (uprev) s -= b * uprev[i];
        y[i] = s;
    }
}

void launch_matvec(const Packed& P, const ColStats& st, const double* v, double* y,
                   const double* beta, const double* uprev, MatvecWork& w, hipStream_t s)
{
    MvGrid g = matvec_grid(P);
    hipLaunchKernelGGL(matvec_kernel, dim3(g.gx, g.gy), dim3(kThreads), 0, s,
                       reinterpret_cast<const uint32_t*>(P.G), P.n, P.p, P.ldp / 4, st.mean,
                       st.inv_sd, v, g.cols_per_split, w.partial, w.counters, y, beta, uprev);
    GKL_LAUNCH_CHECK("matvec_kernel");
}

// ---------------------------------------------------------------------------
// z = A^T u - alpha * vprev
// Block = 4 wavefronts; wavefront w of block x owns individual chunk 4x + w
// (1024 individuals) and keeps its u values in registers across all columns
// of the block's column group.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
rmatvec_kernel(const uint32_t* __restrict__ G, int64_t n, int64_t p, int64_t ldw,
               const double* __restrict__ mean, const double* __restrict__ inv_sd,
               const double* __restrict__ u, int64_t nchunks, double* __restrict__ partial,
               unsigned int* __restrict__ counters, double* __restrict__ z,
               const double* __restrict__ alpha, const double* __restrict__ vprev)
{
    const int lane = threadIdx.x & 63;
    const int64_t chunk = (int64_t)blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
    const int64_t dw = chunk * kWave + lane;
    const int64_t j0 = (int64_t)blockIdx.y * kRCols;
    const int64_t j1 = j0 + kRCols < p ? j0 + kRCols : p;
    if (chunk < nchunks) {
        double uu[kIndPerThread];
#pragma unroll
        for (int k = 0; k < kIndPerThread; ++k) {
            const int64_t i = dw * kIndPerThread + k;
            uu[k] = (dw < ldw && i < n) ? u[i] : 0.0;
        }
        for (int64_t j = j0; j < j1; ++j) {
            const uint32_t word = dw < ldw ? G[j * ldw + dw] : 0xFFFFFFFFu;
            double sg = 0.0, so = 0.0;
#pragma unroll
            for (int k = 0; k < kIndPerThread; ++k) {
                const uint32_t c = (word >> (2 * k)) & 3u;
                const bool obs = c != 3u;
                sg = fma(obs ? (double)c : 0.0, uu[k], sg);
                so += obs ? uu[k] : 0.0;
            }
            sg = wave_sum(sg);
            so = wave_sum(so);
            if (lane == 0) {
                partial[(chunk * p + j) * 2 + 0] = sg;
                partial[(chunk * p + j) * 2 + 1] = so;
            }
        }
    }
    if (!last_block_arrived(&counters[blockIdx.y], gridDim.x)) return;
    const double a = alpha ? *alpha : 0.0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kThreads) {
        double sg = 0.0, so = 0.0;
        for (int64_t c = 0; c < nchunks; ++c) {
            sg += partial[(c * p + j) * 2 + 0];
            so += partial[(c * p + j) * 2 + 1];
        }
        double r = inv_sd[j] * (sg - mean[j] * so);
        if (vprev) r -= a * vprev[j];
        z[j] = r;
    }
}

void launch_rmatvec(const Packed& P, const ColStats& st, const double* u, double* z,
                    const double* alpha, const double* vprev, MatvecWork& w, hipStream_t s)
{
    const int64_t ldw = P.ldp / 4;
    const int64_t nchunks = (ldw + kWave - 1) / kWave;
    dim3 grid(ceil_div(nchunks, kThreads / kWave), ceil_div(P.p, kRCols));
    hipLaunchKernelGGL(rmatvec_kernel, grid, dim3(kThreads), 0, s,
                       reinterpret_cast<const uint32_t*>(P.G), P.n, P.p, ldw, st.mean, st.inv_sd,
                       u, nchunks, w.partial, w.counters, z, alpha, vprev);
    GKL_LAUNCH_CHECK("rmatvec_kernel");
}

}  // namespace gkl
