// Batched Gram-Schmidt, norms and step bookkeeping for many problems (gfx950).
//
// The batched solver runs the FP64 GKL iteration of Section 3 of the paper on
// many genotype matrices at once (one per chromosome, say).  All problems step
// together; every kernel here covers every active problem in one launch
// (grid.y = problem), so one Lanczos step is a fixed sequence of launches that
// is captured once in a HIP graph and replayed.  The step index lives on the
// device (state[0]) for the same reason.
//
// Full reorthogonalisation by classical Gram-Schmidt applied twice (CGS2): for
// a new vector r and basis Q(:, 0:c), h = Q^T r (on the FP64 matrix cores, see
// launch_batch_proj), r <- r - Q h, twice; the norm
// of the result (accumulated while the second update writes r) becomes alpha_j
// or beta_j and r is scaled to unit length.  Sums over row chunks are added in
// chunk order, so results do not depend on scheduling.
#include <math.h>

#include "kernels.h"

namespace gkl {

namespace {
constexpr int kChunk = 2048;       // rows per workgroup in the Gram-Schmidt kernels
constexpr int kPerLane = kChunk / kWave;

struct Side {
    int64_t len;
    int ncols;
    const double* Q;
    double* r;
    double* scalar;
};

__device__ __forceinline__ Side side_of(const BatchDesc& D, int j, int side)
{
    Side s;
    if (side == 0) {
        s.len = D.n;
        s.ncols = j;
        s.Q = D.U;
        s.r = D.U + (int64_t)j * D.n;
        s.scalar = D.alpha + j;
    } else {
        s.len = D.p;
        s.ncols = j + 1;
        s.Q = D.V;
        s.r = D.V + (int64_t)(j + 1) * D.p;
        s.scalar = D.beta + j;
    }
    return s;
}
}  // namespace

size_t bortho_chunks(int64_t len) { return (size_t)((len + kChunk - 1) / kChunk); }

// r <- r - Q h over the chunk's rows; with norm != 0 the chunk's sum of squares
// of the new r goes to npart[chunk].
__global__ void __launch_bounds__(256)
bupdate_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state, int side,
               int norm)
{
    __shared__ double hs[kMaxSvd + 2];
    __shared__ double red[16];
    const BatchDesc& D = desc[blockIdx.y];
    if (!*D.active) return;
    const Side S = side_of(D, state[0], side);
    const int64_t r0 = (int64_t)blockIdx.x * kChunk;
    if (r0 >= S.len) return;
    for (int c = threadIdx.x; c < S.ncols; c += blockDim.x) hs[c] = D.h[c];
    __syncthreads();
    double ss = 0.0;
    for (int t = 0; t < kChunk / 256; ++t) {
        const int64_t row = r0 + threadIdx.x + (int64_t)t * 256;
        if (row >= S.len) break;
        double x = S.r[row];
        for (int c = 0; c < S.ncols; ++c) x = fma(-S.Q[(int64_t)c * S.len + row], hs[c], x);
        S.r[row] = x;
        ss = fma(x, x, ss);
    }
    if (norm) {
        ss = block_sum(ss, red);
        if (threadIdx.x == 0) D.npart[blockIdx.x] = ss;
    }
}

// alpha_j / beta_j = ||r|| from the chunk sums (one wave per problem).  A norm
// at or below 2^-52 sqrt(len) times the largest scalar so far is a breakdown:
// the problem stops (its scalar is 0, the vector is left unscaled and
// *breakdown records the half-step 2j + side, plus one).
__global__ void __launch_bounds__(64)
bnorm_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state, int side)
{
    const BatchDesc& D = desc[blockIdx.x];
    if (!*D.active) return;
    const Side S = side_of(D, state[0], side);
    const int nch = (int)((S.len + kChunk - 1) / kChunk);
    double a = 0.0;
    for (int ch = threadIdx.x; ch < nch; ch += 64) a += D.npart[ch];
    a = wave_sum(a);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(a);
        const double scale = *D.anorm;
        if (!(nrm > 2.220446049250313e-16 * sqrt((double)S.len) * scale) || !(nrm > 0.0)) {
            *S.scalar = 0.0;
            *D.breakdown = 1 + 2 * state[0] + side;   // the half-step, plus one
            *D.active = 0;
        } else {
            *S.scalar = nrm;
            if (nrm > scale) *D.anorm = nrm;
        }
    }
}

__global__ void __launch_bounds__(256)
bscale_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state, int side)
{
    const BatchDesc& D = desc[blockIdx.y];
    if (!*D.active) return;
    const Side S = side_of(D, state[0], side);
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= S.len) return;
    S.r[row] = S.r[row] / *S.scalar;
}

void launch_bortho(const BatchDesc* d, const int* state, int count, int side, int64_t max_len,
                   int hstride, hipStream_t s)
{
    const dim3 gch((unsigned int)bortho_chunks(max_len), (unsigned int)count);
    for (int pass = 0; pass < 2; ++pass) {
        launch_batch_proj(d, state, count, side, hstride, s);
        hipLaunchKernelGGL(bupdate_kernel, gch, dim3(256), 0, s, d, state, side, pass == 1 ? 1 : 0);
        GKL_LAUNCH_CHECK("bupdate_kernel");
    }
    hipLaunchKernelGGL(bnorm_kernel, dim3(count), dim3(64), 0, s, d, state, side);
    GKL_LAUNCH_CHECK("bnorm_kernel");
    hipLaunchKernelGGL(bscale_kernel, dim3(ceil_div(max_len, 256), count), dim3(256), 0, s, d, state,
                       side);
    GKL_LAUNCH_CHECK("bscale_kernel");
}

__global__ void bstep_kernel(int* state)
{
    if (threadIdx.x == 0) state[0] += 1;
}

void launch_bstep(int* state, hipStream_t s)
{
    hipLaunchKernelGGL(bstep_kernel, dim3(1), dim3(64), 0, s, state);
    GKL_LAUNCH_CHECK("bstep_kernel");
}

// Start of a solve: v_0 <- v_0 / ||v_0|| for every active problem (the norm is
// summed in chunk order by one wave per problem).
__global__ void __launch_bounds__(256)
bstart_norm_kernel(const BatchDesc* __restrict__ desc)
{
    __shared__ double red[16];
    const BatchDesc& D = desc[blockIdx.y];
    const int64_t r0 = (int64_t)blockIdx.x * kChunk;
    if (r0 >= D.p) return;
    double ss = 0.0;
    for (int t = 0; t < kChunk / 256; ++t) {
        const int64_t row = r0 + threadIdx.x + (int64_t)t * 256;
        if (row < D.p) ss = fma(D.V[row], D.V[row], ss);
    }
    ss = block_sum(ss, red);
    if (threadIdx.x == 0) D.npart[blockIdx.x] = ss;
}

__global__ void __launch_bounds__(64)
bstart_sum_kernel(const BatchDesc* __restrict__ desc)
{
    const BatchDesc& D = desc[blockIdx.x];
    const int nch = (int)((D.p + kChunk - 1) / kChunk);
    double a = 0.0;
    for (int ch = threadIdx.x; ch < nch; ch += 64) a += D.npart[ch];
    a = wave_sum(a);
    if (threadIdx.x == 0) {
        D.h[0] = sqrt(a);
        *D.anorm = 0.0;
        *D.breakdown = 0;
    }
}

__global__ void __launch_bounds__(256)
bstart_scale_kernel(const BatchDesc* __restrict__ desc)
{
    const BatchDesc& D = desc[blockIdx.y];
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= D.p) return;
    const double nrm = D.h[0];
    D.V[row] = nrm > 0.0 ? D.V[row] / nrm : 0.0;
}

void launch_bstart(const BatchDesc* d, int count, int64_t max_p, int, hipStream_t s)
{
    hipLaunchKernelGGL(bstart_norm_kernel, dim3((unsigned int)bortho_chunks(max_p), count),
                       dim3(256), 0, s, d);
    GKL_LAUNCH_CHECK("bstart_norm_kernel");
    hipLaunchKernelGGL(bstart_sum_kernel, dim3(count), dim3(64), 0, s, d);
    GKL_LAUNCH_CHECK("bstart_sum_kernel");
    hipLaunchKernelGGL(bstart_scale_kernel, dim3(ceil_div(max_p, 256), count), dim3(256), 0, s, d);
    GKL_LAUNCH_CHECK("bstart_scale_kernel");
}


// ---------------------------------------------------------------------------
// Leave-one-block-out (LOCO) batches
// ---------------------------------------------------------------------------
// Problem q is the whole matrix without its SNP block [lohi[2q], lohi[2q+1]):
// its right vectors live in the full p-space with that block's rows zero, so
// A_{-q} v = A v and A_{-q}^T u is A^T u with the block's rows dropped.  The
// products of all problems are then one block product with the whole matrix.

// out[:, q] = v_j (side 0, len = p) or u_j (side 1, len = n) of problem q; zero
// for problems no longer active.
__global__ void __launch_bounds__(256)
loco_gather_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state, int side,
                   double* __restrict__ out, int64_t len)
{
    const int q = blockIdx.y;
    const BatchDesc& D = desc[q];
    const int j = state[0];
    const bool act = *D.active != 0;
    const double* src = side == 0 ? D.V + (int64_t)j * D.p : D.U + (int64_t)j * D.n;
    double* dst = out + (int64_t)q * len;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = act ? src[i] : 0.0;
}

void launch_loco_gather(const BatchDesc* d, const int* state, int count, int side, double* out,
                        int64_t len, hipStream_t s)
{
    unsigned int nb = ceil_div(len, 256);
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(loco_gather_kernel, dim3(nb, count), dim3(256), 0, s, d, state, side, out, len);
    GKL_LAUNCH_CHECK("loco_gather_kernel");
}

// u_j = Y(:, q) - beta_{j-1} u_{j-1}, or - U(:, 0:nlock) rho right after a restart.
__global__ void __launch_bounds__(256)
loco_left_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state,
                 const double* __restrict__ Y, int64_t n)
{
    const BatchDesc& D = desc[blockIdx.y];
    if (!*D.active) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = state[0], nlock = state[1];
    double s = Y[(int64_t)blockIdx.y * n + i];
    if (j > 0 && j == nlock) {
        for (int c = 0; c < nlock; ++c) s -= D.rho[c] * D.U[(int64_t)c * n + i];
    } else if (j > 0) {
        s -= D.beta[j - 1] * D.U[(int64_t)(j - 1) * n + i];
    }
    D.U[(int64_t)j * n + i] = s;
}

void launch_loco_left(const BatchDesc* d, const int* state, int count, const double* Y, int64_t n,
                      hipStream_t s)
{
    hipLaunchKernelGGL(loco_left_kernel, dim3(ceil_div(n, 256), count), dim3(256), 0, s, d, state, Y,
                       n);
    GKL_LAUNCH_CHECK("loco_left_kernel");
}

// v_{j+1} = Z(:, q) with the rows of block q zeroed, - alpha_j v_j.
__global__ void __launch_bounds__(256)
loco_right_kernel(const BatchDesc* __restrict__ desc, const int* __restrict__ state,
                  const double* __restrict__ Z, int64_t p, const int64_t* __restrict__ lohi)
{
    const int q = blockIdx.y;
    const BatchDesc& D = desc[q];
    if (!*D.active) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p) return;
    const int j = state[0];
    const bool own = i >= lohi[2 * q] && i < lohi[2 * q + 1];
    const double z = own ? 0.0 : Z[(int64_t)q * p + i];
    D.V[(int64_t)(j + 1) * p + i] = z - D.alpha[j] * D.V[(int64_t)j * p + i];
}

void launch_loco_right(const BatchDesc* d, const int* state, int count, const double* Z, int64_t p,
                       const int64_t* lohi, hipStream_t s)
{
    hipLaunchKernelGGL(loco_right_kernel, dim3(ceil_div(p, 256), count), dim3(256), 0, s, d, state, Z,
                       p, lohi);
    GKL_LAUNCH_CHECK("loco_right_kernel");
}

// Start vectors: zero the rows of each problem's own block.
__global__ void __launch_bounds__(256)
loco_mask_kernel(const BatchDesc* __restrict__ desc, const int64_t* __restrict__ lohi)
{
    const int q = blockIdx.y;
    const BatchDesc& D = desc[q];
    const int64_t lo = lohi[2 * q], hi = lohi[2 * q + 1];
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
         i += (int64_t)gridDim.x * blockDim.x)
        D.V[i] = 0.0;
}

void launch_loco_mask(const BatchDesc* d, int count, const int64_t* lohi, hipStream_t s)
{
    hipLaunchKernelGGL(loco_mask_kernel, dim3(256, count), dim3(256), 0, s, d, lohi);
    GKL_LAUNCH_CHECK("loco_mask_kernel");
}

}  // namespace gkl
