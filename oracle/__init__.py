"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct FP64 CPU implementation of what the GKL hot
path computes (Chen, Noack & Edelman, "Fast computation of the principal
components of genotype matrices in Julia", arXiv:1808.03374).  Only the test
suite, ``__graft_entry__.smoke()`` and the bench's ``cpu_baseline`` leg may
import it.  It shares no code with the GPU library under
``paper_1808_03374_amd`` and never imports it.

Parity status per function (what pins it is listed in the tests):
  decode, column_stats            pinned (hand-made byte table, closed forms)
  dense_matrix / PackedOperator   pinned (hand-computed column, adjoint, centring,
                                  Frobenius norm from integer counts)
  gkl_svd                         pinned (dense LAPACK SVD, augmented-matrix eigh,
                                  two-group closed form sigma_1 = sqrt(2np),
                                  Frobenius identity at full rank)
  mp_* densities                  pinned (unit mass, Fig. 1 printed edge, Gaussian KS)
  sign_fix                        pinned (hand-made columns with ties and negative
                                  maxima; the left vector flips with the right)
  subspace_angles                 pinned (known rotations from 1.2 down to 1e-9 rad,
                                  orthogonal and identical spans)
  certificate                     pinned (operator with a known SVD: exact triplets,
                                  sigma shifted by known deltas, a tilted vector)
  thick_restart                   pinned (harmonic values and vectors against the
                                  Petrov definition solved as a generalized symmetric
                                  eigenproblem; the restarted relations A V = U H and
                                  A^T U in span of the new right basis, with a dense A)
  gkl_svd_thick                   pinned (dense LAPACK SVD after several restarts of
                                  either kind)
"""
from .gkl_oracle import (  # noqa: F401
    build_library, decode, counts, column_stats, dense_matrix, DenseOperator,
    PackedOperator, cgs2, gkl_svd, GKLResult, sign_fix, certificate,
    thick_restart, gkl_svd_thick, RestartPlan,
    frobenius_sq_from_counts, mp_eigen_density, mp_singular_density,
    mp_singular_edges, subspace_angles,
)
