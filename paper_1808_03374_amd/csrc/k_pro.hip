// Partial reorthogonalisation (PRO) for GKL bidiagonalisation (gfx950, FP64):
// standalone launches of the estimate updates (pro.h holds the updates and the
// description of the method).  The engine uses these only where the new norm
// does not come with the product (the step after a thick restart, whose A v
// also subtracts sum_i rho_i u_i); elsewhere the update runs in the norm kernel
// that follows the product's reduce.
#include "pro.h"

namespace gkl {

namespace {
constexpr int kProThreads = 128;
}  // namespace

__global__ void __launch_bounds__(kProThreads) pro_left_kernel(ProArgs a)
{
    pro_left_body(a, a.alpha[a.j]);
}

__global__ void __launch_bounds__(kProThreads) pro_right_kernel(ProArgs a)
{
    pro_right_body(a, a.beta[a.j]);
}

void launch_pro_left(const ProArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(pro_left_kernel, dim3(1), dim3(kProThreads), 0, s, a);
    GKL_LAUNCH_CHECK("pro_left_kernel");
}

void launch_pro_right(const ProArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(pro_right_kernel, dim3(1), dim3(kProThreads), 0, s, a);
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
