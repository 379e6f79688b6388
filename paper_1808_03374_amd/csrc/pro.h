// Partial reorthogonalisation (PRO): the estimate updates as device functions,
// run by the standalone PRO kernels and by the kernel that turns a product's
// per-workgroup sums of squares into alpha_j or beta_j.
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
//
// Both bodies are run by every thread of one workgroup (blockDim.x a multiple
// of 64, at most 256) and contain barriers.
#pragma once

#include <math.h>

#include "kernels.h"

namespace gkl {

__device__ __forceinline__ double pro_block_max_abs(double v, double* sh)
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

// Row j of mu from row j-1 (in place), given aj = alpha_j.  mu[j-1] is the
// diagonal (1).
__device__ __forceinline__ void pro_left_body(const ProArgs& a, double aj)
{
    __shared__ double sh[4];
    __shared__ int decide;
    const int j = a.j, nlock = a.nlock;
    const ProState& st = a.st;
    const double tau = aj > 0.0 ? a.noise_scale * (*a.norm_est) / aj : a.noise_scale;
    const double bprev = j > 0 ? a.beta[j - 1] : 0.0;
    double local = 0.0;
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
        const double nu_i = st.nu[i];
        const double nu_i1 = (i + 1 == j) ? 1.0 : st.nu[i + 1];
        double vAu;
        if (i < nlock) vAu = a.theta[i] * nu_i + a.rho[i] * ((nlock == j) ? 1.0 : st.nu[nlock]);
        else vAu = a.alpha[i] * nu_i + a.beta[i] * nu_i1;
        const double mu_old = (i == j - 1) ? 1.0 : st.mu[i];
        double m = aj > 0.0 ? (vAu - bprev * mu_old) / aj : 0.0;
        m += (m >= 0.0 ? tau : -tau);
        st.mu[i] = m;
        local = fmax(local, fabs(m));
    }
    const double mx = pro_block_max_abs(local, sh);
    if (threadIdx.x == 0) {
        int f = 0;
        if (st.force[0] > 0) { f = 1; st.force[0] -= 1; }
        if (mx > a.omega) { f = 1; st.force[0] = st.force[0] > 1 ? st.force[0] : 1; }
        *st.flag_left = f;
        decide = f;
    }
    __syncthreads();
    if (decide)
        for (int i = threadIdx.x; i < j; i += blockDim.x) st.mu[i] = a.noise_scale;
}

// Row j+1 of nu from row j (in place), given bj = beta_j; mu holds row j,
// mu[j] is the diagonal.
__device__ __forceinline__ void pro_right_body(const ProArgs& a, double bj)
{
    __shared__ double sh[4];
    __shared__ double rho_mu;
    __shared__ int decide;
    const int j = a.j, nlock = a.nlock;
    const ProState& st = a.st;
    const double aj = a.alpha[j];
    const double tau = bj > 0.0 ? a.noise_scale * (*a.norm_est) / bj : a.noise_scale;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < nlock; ++t) s += a.rho[t] * st.mu[t];
        rho_mu = s;
    }
    __syncthreads();
    double local = 0.0;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        const double mu_i = (i == j) ? 1.0 : st.mu[i];
        double uAv;
        if (i < nlock) {
            uAv = a.theta[i] * mu_i;
        } else if (i == nlock && nlock > 0) {
            uAv = a.alpha[i] * mu_i + rho_mu;
        } else {
            uAv = a.alpha[i] * mu_i + (i > 0 ? a.beta[i - 1] * st.mu[i - 1] : 0.0);
        }
        const double nu_old = (i == j) ? 1.0 : st.nu[i];
        double v = bj > 0.0 ? (uAv - aj * nu_old) / bj : 0.0;
        v += (v >= 0.0 ? tau : -tau);
        st.nu[i] = v;
        local = fmax(local, fabs(v));
    }
    const double mx = pro_block_max_abs(local, sh);
    if (threadIdx.x == 0) {
        int f = 0;
        if (st.force[1] > 0) { f = 1; st.force[1] -= 1; }
        if (mx > a.omega) { f = 1; st.force[1] = st.force[1] > 1 ? st.force[1] : 1; }
        *st.flag_right = f;
        decide = f;
    }
    __syncthreads();
    if (decide)
        for (int i = threadIdx.x; i <= j; i += blockDim.x) st.nu[i] = a.noise_scale;
}

// Norm of a product's output from the sums of squares its reduce kernel left
// in npart[0 .. nparts) (one per workgroup): summed in index order by one
// workgroup, ||y|| goes to *nrm_out and, with pro = 1 (left) or 2 (right),
// the PRO update for that norm follows.
__device__ __forceinline__ void norm_pro_body(const NormTail& t, int nparts)
{
    __shared__ double red[16];
    double a = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) a += t.npart[b];
    const double nrm = sqrt(block_sum(a, red));
    if (threadIdx.x == 0) *t.nrm_out = nrm;
    if (t.pro == 1) pro_left_body(t.pa, nrm);
    else if (t.pro == 2) pro_right_body(t.pa, nrm);
}

}  // namespace gkl
