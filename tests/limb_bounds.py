"""Error bound of the FP64 products formed in int8 limbs (shared by the GPU tests).

The vector is scaled by a power of two 2^e below twice its largest magnitude
(for A v: of (3 - mu_j) s_j v_j, which bounds s_j v_j) and rounded to a 52-bit
integer, so every entry moves by at most 2^-53 2^e; the limb sums are exact.
Per output element the quantisation therefore contributes at most
2^-53 2^e (sum_j |c_ij| + sum_j m_ij |mu_j - 3|) <= 2^-52 max|scaled| 6 p (A v)
and s_j 2^-52 max|u| 6 n (A^T u), codes c <= 3.  It shows where a product
cancels to (near) zero: the quantised s_j v_j times c_ij no longer cancels the
exact mean term mu_j s_j v_j to the last bit.
"""
import numpy as np

import oracle


def quantisation_slack(g, v, u):
    """Norm-wise bounds (for A v, for A^T u) of the quantisation error."""
    st = oracle.column_stats(g.n, *oracle.counts(g.packed, g.n, g.p))
    w = np.max(np.abs((3.0 - st.mean) * st.inv_sd * v), initial=0.0)
    sy = np.sqrt(g.n) * 2.0 ** -52 * w * 6 * g.p
    sz = np.sqrt(g.p) * 2.0 ** -52 * np.max(np.abs(u), initial=0.0) * 6 * g.n * np.max(st.inv_sd)
    return sy, sz
