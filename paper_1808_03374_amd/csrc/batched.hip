// Batched persistent solver -- entry points (built in a later step).
#include "engine.h"

namespace gkl {
struct BatchState {};
void destroy_batch(BatchState* b) { delete b; }
}  // namespace gkl

extern "C" {
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
