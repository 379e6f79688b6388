"""Pins of the oracle's thick restart (Section 3, "Thick restarting").

The harmonic restart is checked against the definition of harmonic Ritz pairs
solved by a generic routine, and both restart kinds against the relations a
restarted Golub-Kahan-Lanczos decomposition must satisfy, with a dense matrix.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle.gkl_oracle as og
import synth


def _matrix(n=150, p=400, seed=11):
    g = synth.config("c2", n=n, p=p, seed=seed)
    st = og.column_stats(g.n, *og.counts(g.packed, g.n, g.p))
    return og.dense_matrix(og.decode(g.packed, g.n, g.p), st.mean, st.inv_sd)


def _decomposition(A, m, seed=3):
    """m plain GKL steps with full reorthogonalisation (test-side, numpy):
    A V_m = U_m B, A^T U_m = V_m B^T + beta v_{m+1} e_m^T."""
    n, p = A.shape
    U = np.zeros((n, m))
    V = np.zeros((p, m + 1))
    B = np.zeros((m, m))
    v = np.random.default_rng(seed).standard_normal(p)
    V[:, 0] = v / np.linalg.norm(v)
    beta = 0.0
    for j in range(m):
        w = A @ V[:, j] - (beta * U[:, j - 1] if j else 0.0)
        for _ in range(2):
            w -= U[:, :j] @ (U[:, :j].T @ w)
        a = np.linalg.norm(w)
        U[:, j] = w / a
        B[j, j] = a
        r = A.T @ U[:, j] - a * V[:, j]
        for _ in range(2):
            r -= V[:, : j + 1] @ (V[:, : j + 1].T @ r)
        beta = np.linalg.norm(r)
        V[:, j + 1] = r / beta
        if j + 1 < m:
            B[j, j + 1] = beta
    return U, V, B, beta


def _harmonic_by_definition(A, V, m):
    """Harmonic Ritz pairs of M = A^T A on span(V_m): x = V_m y with
    M x - theta x orthogonal to M V_m, i.e. (M V)^T (M V) y = theta (M V)^T V y.
    With M V = Q R (R invertible) that is R y = theta Q^T V y, solved here as the
    generalized eigenproblem Q^T V y = mu R y, theta = 1 / mu (no squaring of M V)."""
    Vm = V[:, :m]
    Q, R = np.linalg.qr(A.T @ (A @ Vm))
    mu, Y = scipy.linalg.eig(Q.T @ Vm, R)
    theta = 1.0 / mu.real
    order = np.argsort(theta)[::-1]
    return theta[order], Vm @ Y[:, order].real


def _angles(X, Y):
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    s = np.linalg.svd(qy - qx @ (qx.T @ qy), compute_uv=False)
    return np.arcsin(np.clip(s, 0.0, 1.0))


def harmonic_definition_pin(m=24, l=10):
    # a tall matrix: full column rank, so B_m is well conditioned and the
    # definition's solution is accurate to the tolerance below
    A = _matrix(400, 150)
    U, V, B, beta = _decomposition(A, m)
    plan = og.thick_restart(B, beta, l, "harmonic")
    theta, X = _harmonic_by_definition(A, V, m)
    ok_values = np.allclose(plan.values ** 2, theta[:l], rtol=1e-10, atol=0)
    Vn = V @ plan.Z
    ok_vectors = _angles(X[:, :l], Vn[:, :l]).max() < 1e-8
    return bool(ok_values and ok_vectors)


def relations_pin(kind, shape=(400, 150), tol=1e-12, m=24, l=10):
    A = _matrix(*shape)
    U, V, B, beta = _decomposition(A, m)
    plan = og.thick_restart(B, beta, l, kind)
    Un = U @ plan.Yl
    Vn = V @ plan.Z
    scale = np.linalg.norm(A, 2)
    ok_orth = (np.abs(Un.T @ Un - np.eye(l)).max() < 1e-12
               and np.abs(Vn.T @ Vn - np.eye(l + 1)).max() < 1e-12)
    # A V_new[:, :l] = U_new H
    ok_left = np.linalg.norm(A @ Vn[:, :l] - Un @ plan.H) <= tol * scale
    # A^T U_new lies in span(V_new) with coefficients [H^T; c^T]
    M = np.vstack([plan.H.T, plan.c[None, :]])
    ok_right = np.linalg.norm(A.T @ Un - Vn @ M) <= tol * scale
    # the coupling is what the next step's A v_l has along U_new
    ok_c = np.allclose(Un.T @ (A @ Vn[:, l]), plan.c, rtol=0, atol=1e-12 * scale)
    return bool(ok_orth and ok_left and ok_right and ok_c)


def thick_solve_pin(kind, k=6, m=20, l=12):
    A = _matrix(200, 500, 5)
    op = og.DenseOperator(A)
    res = og.gkl_svd_thick(op, k, 1e-12, m, l, kind, v0=synth.start_vector(500, 2))
    s = np.linalg.svd(A, compute_uv=False)[:k]
    ok_sigma = res.converged and np.all(np.abs(res.sigma - s) <= 1e-10 * s[0])
    R = A @ res.V - res.U * res.sigma
    ok_vec = np.linalg.norm(R, axis=0).max() <= 1e-9 * s[0]
    return bool(ok_sigma and ok_vec and res.restarts >= 2)


def test_harmonic_values_and_vectors_match_the_definition():
    assert harmonic_definition_pin()


def test_ritz_values_are_not_the_harmonic_ones():
    # the two kinds keep different vectors (else the definition pin proves little)
    A = _matrix()
    U, V, B, beta = _decomposition(A, 24)
    h = og.thick_restart(B, beta, 10, "harmonic")
    r = og.thick_restart(B, beta, 10, "ritz")
    assert np.abs(h.values - r.values).max() > 1e-6 * r.values[0]
    assert _angles(V @ h.Z[:, :10], V @ r.Z[:, :10]).max() > 1e-6


# Tall: full column rank, B well conditioned.  Wide: the Krylov space closes in
# on a null vector of A and B's smallest singular value falls to about 1e-6 of
# its largest; the restart must not go through B^-1 there (it would carry that
# condition number into the relations), so the same bound applies.
@pytest.mark.parametrize("shape,tol", [((400, 150), 1e-12), ((150, 400), 1e-12)])
@pytest.mark.parametrize("kind", ["ritz", "harmonic"])
def test_restart_relations(kind, shape, tol):
    assert relations_pin(kind, shape, tol)


def test_ritz_restart_head_is_diagonal():
    # ordinary restart: H = diag(sigma), c = beta P(m, :l) (Wu & Simon)
    A = _matrix()
    U, V, B, beta = _decomposition(A, 24)
    plan = og.thick_restart(B, beta, 10, "ritz")
    P, S, _ = np.linalg.svd(B)
    assert np.allclose(plan.H, np.diag(S[:10]), atol=1e-12 * S[0])
    assert np.allclose(plan.c, beta * P[-1, :10], atol=1e-12 * S[0])


@pytest.mark.parametrize("kind", ["ritz", "harmonic"])
def test_thick_restarted_solve_matches_lapack(kind):
    assert thick_solve_pin(kind)


# ---------------------------------------------------------------------------
# Planted mistakes: each variant of thick_restart must fail a pin above
# ---------------------------------------------------------------------------

def _variant(mistake):
    def restart(B, beta_m, l, kind):
        m = B.shape[0]
        em = np.zeros(m)
        em[m - 1] = 1.0
        if kind == "ritz":
            P, S, Qt = np.linalg.svd(B)
            Yl = P[:, :l]
            Z = np.zeros((m + 1, l + 1))
            Z[:m, :l] = Qt.T[:, :l]
            Z[m, l] = 1.0
            values = S[:l].copy()
        else:
            if mistake == "svd_of_B":
                Ph, Sh, Qt = np.linalg.svd(B)
                Qht = np.zeros((m + 1, m + 1))
                Qht[:m, :m] = Qt
                Qht[m, m] = 1.0
            else:
                Ph, Sh, Qht = np.linalg.svd(np.hstack([B, beta_m * em[:, None]]))
            Yl = Ph[:, :l]
            last = np.eye(m + 1)[m] if mistake == "null_is_v_next" else Qht[m]
            QS = np.hstack([Qht[:l].T, last[:, None]])
            r = QS[m, :]
            v = r.copy()
            v[l] += np.copysign(np.linalg.norm(r), r[l])
            Z = QS - np.outer(QS @ v, (2.0 / (v @ v)) * v)
            Z[m, :l] = 0.0
            values = Sh[:l].copy()
        H = Yl.T @ B @ Z[:m, :l]
        c = Yl.T @ B @ Z[:m, l]
        if mistake != "c_without_v_next":
            c = c + Z[m, l] * beta_m * Yl[m - 1, :]
        if mistake == "c_sign":
            c = -c
        return og.RestartPlan(Yl, Z, H, c, values)
    return restart


def test_variant_without_mistake_passes(monkeypatch):
    monkeypatch.setattr(og, "thick_restart", _variant(None))
    assert harmonic_definition_pin()
    assert relations_pin("harmonic") and relations_pin("ritz")


def test_svd_of_B_instead_of_the_augmented_matrix_is_caught(monkeypatch):
    monkeypatch.setattr(og, "thick_restart", _variant("svd_of_B"))
    assert not harmonic_definition_pin()


def test_dropping_the_harmonic_residual_direction_is_caught(monkeypatch):
    monkeypatch.setattr(og, "thick_restart", _variant("null_is_v_next"))
    assert not relations_pin("harmonic")


def test_coupling_without_the_next_vector_term_is_caught(monkeypatch):
    monkeypatch.setattr(og, "thick_restart", _variant("c_without_v_next"))
    assert not relations_pin("ritz")
    assert not relations_pin("harmonic")


def test_coupling_sign_is_caught(monkeypatch):
    monkeypatch.setattr(og, "thick_restart", _variant("c_sign"))
    assert not relations_pin("ritz")
    assert not thick_solve_pin("ritz")


@pytest.mark.parametrize("kind", ["ritz", "harmonic"])
def test_first_cycle_is_the_plain_recurrence(kind):
    # before its first restart the restarted run is plain GKL from the same start
    A = _matrix(200, 500, 5)
    v0 = synth.start_vector(500, 2)
    thick = og.gkl_svd_thick(og.DenseOperator(A), 6, 1e-12, 20, 12, kind, v0=v0)
    plain = og.gkl_svd(og.DenseOperator(A), 6, tol=1e-30, v0=v0, max_steps=20)
    assert np.allclose(thick.alphas[:20], plain.alphas, rtol=1e-13, atol=0)
    assert np.allclose(thick.betas[:20], plain.betas, rtol=1e-13, atol=0)
    # and the run did restart (the later scalars come from the restarted basis)
    assert thick.restarts >= 1 and len(thick.alphas) > 20
