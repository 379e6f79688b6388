"""MI355X (gfx950) Golub-Kahan-Lanczos PCA of 2-bit packed genotype matrices.

Thin Python binding over the C ABI in include/gkl.h (libgkl.so).  The binding
only marshals arguments: every step of the computation runs in the library's
HIP kernels.  PyTorch is used for device memory and streams.  If the compiled
library is missing, importing the binding raises -- there is no fallback.

Method: Chen, Noack & Edelman, arXiv:1808.03374 (Section 3: GKL
bidiagonalisation with thick restart and full or partial reorthogonalisation).
"""
from ._binding import (  # noqa: F401
    GKL_OK, GKL_ERR_INVALID, GKL_ERR_NOMEM, GKL_ERR_DEVICE, GKL_NOT_CONVERGED,
    GKL_ERR_BREAKDOWN, GKL_ERR_INTERNAL, GKL_ERR_UNSUPPORTED, GKL_REORTH_FULL,
    GKL_REORTH_PARTIAL, GKL_REORTH_ONESIDED, GKL_PREC_FP64, GKL_PREC_MIXED, GKL_PREC_MIXED_INT8, GKL_PREC_BLOCK_FP64,
    GKL_FP64_AUTO, GKL_FP64_LUT, GKL_FP64_LIMBS, GKL_FP64_LUT_LIMBS, GKL_TRACE_FIELDS, GKLError,
    GKL_RESTART_RITZ, GKL_RESTART_HARMONIC,
    gkl_options, gkl_info, lib, library_path, gkl_options_default, gkl_status_string,
    gkl_last_error, gkl_create, gkl_create_ex, gkl_solve, gkl_destroy, gkl_create_batched,
    gkl_solve_batched, gkl_create_loco, gkl_column_stats, gkl_unpack, gkl_matvec, gkl_rmatvec,
    gkl_matmat_mixed, gkl_rmatmat_mixed, gkl_get_trace, gkl_dense_svd, gkl_dense_svd_noalloc, gkl_read_rate, gkl_batched_plan,
    Context, BatchedContext, LocoContext, solve, declared_functions,
)
