"""Oracle pins: the implicit operator and the plain GKL solver.

Pins used (none of them re-types the oracle's own formulas):
  * adjoint and centring identities of the operator;
  * the plain C packed operator against a dense NumPy matrix (two independent routes);
  * dense LAPACK SVD of the explicit matrix, and the eigenvalues of the augmented
    matrix [0 A; A^T 0] (Section 4, ARPACK paragraph) via a symmetric eigensolver;
  * the two-group closed form sigma_1 = sqrt(2 n p), which also fixes the scaling
    convention 1/sqrt(2 f (1 - f));
  * sum sigma_i^2 = ||A||_F^2 at full rank (Frobenius norm from integer counts);
  * Krylov invariants: orthonormal bases and centred scores.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
import synth


def _problem(name, n, p, seed=None):
    g = synth.config(name, n=n, p=p, seed=seed)
    st = oracle.column_stats(g.n, *oracle.counts(g.packed, g.n, g.p))
    codes = oracle.decode(g.packed, g.n, g.p)
    A = oracle.dense_matrix(codes, st.mean, st.inv_sd)
    return g, st, A


def test_operator_adjoint_and_centring():
    g, st, A = _problem("c2", 300, 900)
    op = oracle.PackedOperator(g.packed, g.n, g.p, st)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(g.p)
    u = rng.standard_normal(g.n)
    Av = op.matvec(v)
    Atu = op.rmatvec(u)
    scale = np.linalg.norm(Av) * np.linalg.norm(u)
    assert abs(u @ Av - Atu @ v) <= 1e-12 * scale
    # columns are centred over observed entries, so the scores sum to zero
    assert abs(np.sum(Av)) <= 1e-12 * np.sum(np.abs(A)) * np.max(np.abs(v))


def test_packed_operator_matches_dense():
    g, st, A = _problem("c1", 257, 611)
    op = oracle.PackedOperator(g.packed, g.n, g.p, st)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(g.p)
    u = rng.standard_normal(g.n)
    assert np.allclose(op.matvec(v), A @ v, rtol=0, atol=1e-12 * np.linalg.norm(A @ v))
    assert np.allclose(op.rmatvec(u), A.T @ u, rtol=0, atol=1e-12 * np.linalg.norm(A.T @ u))
    rows = np.array([0, 5, 256, 100])
    cols = np.array([610, 0, 3])
    assert np.allclose(op.matvec_rows(v, rows), (A @ v)[rows], rtol=1e-13, atol=1e-13)
    assert np.allclose(op.rmatvec_cols(u, cols), (A.T @ u)[cols], rtol=1e-13, atol=1e-13)


def _check_against_dense(A, res, k, rel=1e-10):
    s_ref = np.linalg.svd(A, compute_uv=False)[:k]
    assert np.all(np.abs(res.sigma - s_ref) <= rel * s_ref[0])
    return s_ref


@pytest.mark.parametrize("name,n,p", [("c1", 300, 800), ("c2", 400, 300), ("c5", 250, 2500)])
def test_gkl_matches_dense_svd(name, n, p):
    g, st, A = _problem(name, n, p)
    k = 10
    res = oracle.gkl_svd(oracle.DenseOperator(A), k, tol=1e-12,
                         v0=synth.start_vector(p, 7))
    assert res.converged
    _check_against_dense(A, res, k)
    # orthonormality and centring of the returned vectors
    assert np.abs(res.U.T @ res.U - np.eye(k)).max() < 1e-12
    assert np.abs(res.V.T @ res.V - np.eye(k)).max() < 1e-12
    assert np.abs(res.U.sum(axis=0)).max() < 1e-10
    # A V = U S to the residual tolerance
    R = A @ res.V - res.U * res.sigma
    assert np.linalg.norm(R, axis=0).max() <= 1e-10 * res.sigma[0]


def test_gkl_matches_augmented_eigenvalues():
    g, st, A = _problem("c1", 120, 200)
    n, p = A.shape
    H = np.zeros((n + p, n + p))
    H[:n, n:] = A
    H[n:, :n] = A.T
    ev = scipy.linalg.eigh(H, eigvals_only=True)
    k = 8
    res = oracle.gkl_svd(oracle.PackedOperator(g.packed, n, p, st), k, tol=1e-12,
                         v0=synth.start_vector(p, 3))
    top = ev[::-1][:k]
    bottom = -ev[:k]
    assert np.allclose(res.sigma, top, rtol=0, atol=1e-10 * top[0])
    assert np.allclose(res.sigma, bottom, rtol=0, atol=1e-10 * top[0])


def test_gkl_full_small_config_against_lapack():
    g, st, A = _problem("c1", 1000, 5000)
    k = 10
    op = oracle.PackedOperator(g.packed, g.n, g.p, st)
    res = oracle.gkl_svd(op, k, tol=1e-12, v0=synth.start_vector(g.p, 1))
    assert res.converged
    Uref, s_ref, Vt = np.linalg.svd(A, full_matrices=False)
    assert np.all(np.abs(res.sigma - s_ref[:k]) <= 1e-10 * s_ref[0])
    # the leading, well separated singular vector agrees up to sign
    ang = oracle.subspace_angles(res.V[:, :1], Vt[:1].T)
    assert ang.max() < 1e-8


def test_two_group_closed_form():
    # individuals 0..n/2-1 carry code 0 in every SNP, the rest code 2: mu = 1,
    # f = 1/2, s = sqrt 2, A = sqrt2 * sgn 1^T, so sigma_1 = sqrt(2 n p) exactly.
    n, p = 40, 30
    codes = np.zeros((n, p), dtype=np.int64)
    codes[n // 2:] = 2
    packed = synth.pack_codes(codes)
    op = oracle.PackedOperator(packed, n, p)
    res = oracle.gkl_svd(op, 1, tol=1e-13, v0=synth.start_vector(p, 0),
                         spare_left=synth.spare_directions(n, 4, 0),
                         spare_right=synth.spare_directions(p, 4, 0))
    assert abs(res.sigma[0] - np.sqrt(2.0 * n * p)) <= 1e-12 * np.sqrt(2.0 * n * p)
    # the scores separate the groups
    assert np.all(np.sign(res.U[: n // 2, 0]) == -np.sign(res.U[n // 2:, 0]))


def test_full_rank_frobenius_identity():
    g, st, A = _problem("c1", 7, 9)
    r = np.linalg.matrix_rank(A)
    res = oracle.gkl_svd(oracle.PackedOperator(g.packed, 7, 9, st), r, tol=1e-13,
                         v0=synth.start_vector(9, 5), spare_left=synth.spare_directions(7, 8, 1),
                         spare_right=synth.spare_directions(9, 8, 1))
    assert abs(np.sum(res.sigma ** 2) - oracle.frobenius_sq_from_counts(st)) <= 1e-12 * np.sum(
        res.sigma ** 2)


def test_gkl_step_scalars_invariant():
    # A V_j = U_j B_j holds along the run (plain GKL, no restart)
    g, st, A = _problem("c2", 200, 500)
    res = oracle.gkl_svd(oracle.DenseOperator(A), 5, tol=1e-14, max_steps=25,
                         v0=synth.start_vector(500, 9))
    assert res.steps == 25 and np.all(res.alphas > 0) and np.all(res.betas > 0)
