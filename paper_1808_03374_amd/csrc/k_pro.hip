// Partial reorthogonalisation (PRO) for GKL bidiagonalisation (gfx950, FP64).
//
// Section 3 of the paper, "Choice of reorthogonalization strategy", offers
// partial reorthogonalisation (Simon 1984; Larsen 1998) with a threshold omega
// (1e-8 in its experiments).  The loss of orthogonality is not measured but
// estimated by recurrences derived from the two GKL relations
//     A v_i   = alpha_i u_i + beta_{i-1} u_{i-1}
//     A^T u_i = alpha_i v_i + beta_i v_{i+1}
// (after a thick restart the first l relations become A v_i = theta_i u_i and
// A^T u_i = theta_i v_i + rho_i v_l, and A v_l gains sum_i rho_i u_i):
//   alpha_j mu_{j,i}    = v_j^T A^T u_i - beta_{j-1} mu_{j-1,i}
//   beta_j  nu_{j+1,i}  = u_j^T A v_i   - alpha_j  nu_{j,i}
// with mu_{j,i} ~ u_j^T u_i and nu_{j,i} ~ v_j^T v_i.  Each update adds a
// rounding-noise term of the same sign.  When an estimate exceeds omega the
// new vector is reorthogonalised against its whole basis, and so is the next
// vector on the same side (Simon's rule); the estimates of a reorthogonalised
// vector are reset to the noise level.  Estimates live in device memory so a
// step needs no host round trip.
#include <math.h>

#include "kernels.h"

namespace gkl {

namespace {
constexpr int kProThreads = 128;

__device__ __forceinline__ double block_max_abs(double v, double* sh)
{
    v = fabs(v);
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) m = fmax(m, sh[w]);
    return m;
}
}  // namespace

// Row j of mu from row j-1 (in place).  mu[j-1] is the diagonal (1).
__global__ void __launch_bounds__(kProThreads)
pro_left_kernel(const double* __restrict__ alpha, const double* __restrict__ beta,
                const double* __restrict__ theta, const double* __restrict__ rho, int nlock, int j,
                double omega, double noise_scale, const double* __restrict__ norm_est,
                ProState st)
{
    __shared__ double sh[4];
    const double aj = alpha[j];
    const double tau = aj > 0.0 ? noise_scale * (*norm_est) / aj : noise_scale;
    const double bprev = j > 0 ? beta[j - 1] : 0.0;
    double local = 0.0;
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
        const double nu_i = st.nu[i];
        const double nu_i1 = (i + 1 == j) ? 1.0 : st.nu[i + 1];
        double vAu;
        if (i < nlock) vAu = theta[i] * nu_i + rho[i] * ((nlock == j) ? 1.0 : st.nu[nlock]);
        else vAu = alpha[i] * nu_i + beta[i] * nu_i1;
        const double mu_old = (i == j - 1) ? 1.0 : st.mu[i];
        double m = aj > 0.0 ? (vAu - bprev * mu_old) / aj : 0.0;
        m += (m >= 0.0 ? tau : -tau);
        st.mu[i] = m;
        local = fmax(local, fabs(m));
    }
    const double mx = block_max_abs(local, sh);
    __shared__ int decide;
    if (threadIdx.x == 0) {
        int f = 0;
        if (st.force[0] > 0) { f = 1; st.force[0] -= 1; }
        if (mx > omega) { f = 1; st.force[0] = st.force[0] > 1 ? st.force[0] : 1; }
        *st.flag_left = f;
        decide = f;
    }
    __syncthreads();
    if (decide)
        for (int i = threadIdx.x; i < j; i += blockDim.x) st.mu[i] = noise_scale;
}

// Row j+1 of nu from row j (in place); mu holds row j, mu[j] is the diagonal.
__global__ void __launch_bounds__(kProThreads)
pro_right_kernel(const double* __restrict__ alpha, const double* __restrict__ beta,
                 const double* __restrict__ theta, const double* __restrict__ rho, int nlock, int j,
                 double omega, double noise_scale, const double* __restrict__ norm_est,
                 ProState st)
{
    __shared__ double sh[4];
    __shared__ double rho_mu;
    const double aj = alpha[j];
    const double bj = beta[j];
    const double tau = bj > 0.0 ? noise_scale * (*norm_est) / bj : noise_scale;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < nlock; ++t) s += rho[t] * st.mu[t];
        rho_mu = s;
    }
    __syncthreads();
    double local = 0.0;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        const double mu_i = (i == j) ? 1.0 : st.mu[i];
        double uAv;
        if (i < nlock) {
            uAv = theta[i] * mu_i;
        } else if (i == nlock && nlock > 0) {
            uAv = alpha[i] * mu_i + rho_mu;
        } else {
            uAv = alpha[i] * mu_i + (i > 0 ? beta[i - 1] * st.mu[i - 1] : 0.0);
        }
        const double nu_old = (i == j) ? 1.0 : st.nu[i];
        double v = bj > 0.0 ? (uAv - aj * nu_old) / bj : 0.0;
        v += (v >= 0.0 ? tau : -tau);
        st.nu[i] = v;
        local = fmax(local, fabs(v));
    }
    const double mx = block_max_abs(local, sh);
    __shared__ int decide;
    if (threadIdx.x == 0) {
        int f = 0;
        if (st.force[1] > 0) { f = 1; st.force[1] -= 1; }
        if (mx > omega) { f = 1; st.force[1] = st.force[1] > 1 ? st.force[1] : 1; }
        *st.flag_right = f;
        decide = f;
    }
    __syncthreads();
    if (decide)
        for (int i = threadIdx.x; i <= j; i += blockDim.x) st.nu[i] = noise_scale;
}

void launch_pro_left(const double* alpha, const double* beta, const double* theta,
                     const double* rho, int nlock, int j, double omega, double noise_scale,
                     const double* norm_est, const ProState& st, hipStream_t s)
{
    hipLaunchKernelGGL(pro_left_kernel, dim3(1), dim3(kProThreads), 0, s, alpha, beta, theta, rho,
                       nlock, j, omega, noise_scale, norm_est, st);
    GKL_LAUNCH_CHECK("pro_left_kernel");
}

void launch_pro_right(const double* alpha, const double* beta, const double* theta,
                      const double* rho, int nlock, int j, double omega, double noise_scale,
                      const double* norm_est, const ProState& st, hipStream_t s)
{
    hipLaunchKernelGGL(pro_right_kernel, dim3(1), dim3(kProThreads), 0, s, alpha, beta, theta,
                       rho, nlock, j, omega, noise_scale, norm_est, st);
    GKL_LAUNCH_CHECK("pro_right_kernel");
}

__global__ void pro_reset_kernel(ProState st, int maxm, int force)
{
    for (int i = threadIdx.x; i < maxm + 1; i += blockDim.x) {
        if (i < maxm) st.mu[i] = 0.0;
        st.nu[i] = 0.0;
    }
    if (threadIdx.x == 0) {
        st.force[0] = force;
        st.force[1] = force;
        *st.flag_left = 1;
        *st.flag_right = 1;
    }
}

void launch_pro_reset(const ProState& st, int maxm, int force, hipStream_t s)
{
    hipLaunchKernelGGL(pro_reset_kernel, dim3(1), dim3(256), 0, s, st, maxm, force);
    GKL_LAUNCH_CHECK("pro_reset_kernel");
}

}  // namespace gkl
