// Blocked mixed-precision GKL (split-BF16 MFMA products) -- placeholder until built.
#include "engine.h"

namespace gkl {
struct MixedState {};
struct BatchState {};
bool mixed_supported() { return false; }
void destroy_mixed(MixedState* m) { delete m; }
void destroy_batch(BatchState* b) { delete b; }
}  // namespace gkl

void gkl_ctx::setup_mixed() { gkl::fail(GKL_ERR_UNSUPPORTED, "mixed precision path not built"); }
gkl_status gkl_ctx::solve_mixed(double*, double*, int64_t, double*, int64_t)
{
    gkl::fail(GKL_ERR_UNSUPPORTED, "mixed precision path not built");
}

extern "C" {
gkl_status gkl_matmat_mixed(gkl_ctx*, const double*, int32_t, double*) { return GKL_ERR_UNSUPPORTED; }
gkl_status gkl_rmatmat_mixed(gkl_ctx*, const double*, int32_t, double*) { return GKL_ERR_UNSUPPORTED; }
gkl_status gkl_create_batched(int32_t, const uint8_t* const*, const int64_t*, const int64_t*, int32_t,
                              double, int32_t, const gkl_options*, gkl_ctx**)
{
    return GKL_ERR_UNSUPPORTED;
}
gkl_status gkl_solve_batched(gkl_ctx*, double* const*, double* const*, const int64_t*, double* const*,
                             const int64_t*, gkl_info*)
{
    return GKL_ERR_UNSUPPORTED;
}
}
