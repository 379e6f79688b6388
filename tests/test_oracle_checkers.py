"""Pins of the oracle's checking functions: the sign rule, principal angles and
the residual certificate.  Each is fed inputs whose answer is known in closed
form, and a planted mistake in each is shown to fail its pin."""
import numpy as np
import pytest

import oracle
import oracle.gkl_oracle as og


# ---------------------------------------------------------------------------
# sign rule: largest-|.| entry of each right vector positive, lowest index on
# ties, the left vector flipped with it
# ---------------------------------------------------------------------------

def _sign_case():
    V = np.array([[0.1, 0.5, -0.3],
                  [-0.9, -0.5, 0.2],
                  [0.3, 0.1, 0.3],
                  [0.2, -0.5, -0.3]])
    U = np.array([[1.0, 2.0, 3.0],
                  [-4.0, 5.0, -6.0]])
    # column 0: largest |.| is -0.9 (row 1) -> flip
    # column 1: |.| ties at 0.5 in rows 0, 1, 3; the lowest index (0, +0.5) decides -> keep
    #           (the highest, row 3, holds -0.5)
    # column 2: |.| ties at 0.3 in rows 0, 2, 3; row 0 holds -0.3 -> flip
    flips = np.array([-1.0, 1.0, -1.0])
    return U, V, flips


def _sign_pin():
    U, V, flips = _sign_case()
    U2, V2 = og.sign_fix(U, V)
    return bool(np.array_equal(V2, V * flips) and np.array_equal(U2, U * flips))


def test_sign_fix_closed_cases():
    assert _sign_pin()
    U, V, flips = _sign_case()
    U2, V2 = oracle.sign_fix(U, V)
    for i in range(V.shape[1]):
        first = int(np.flatnonzero(np.abs(V2[:, i]) == np.abs(V2[:, i]).max())[0])
        assert V2[first, i] > 0
    # the inputs are left untouched and applying the rule twice changes nothing
    assert np.array_equal(V, _sign_case()[1])
    U3, V3 = og.sign_fix(U2, V2)
    assert np.array_equal(U3, U2) and np.array_equal(V3, V2)


def test_sign_fix_that_forgets_u_is_caught(monkeypatch):
    def wrong(U, V):
        V = V.copy()
        for i in range(V.shape[1]):
            idx = int(np.argmax(np.abs(V[:, i])))
            if V[idx, i] < 0:
                V[:, i] = -V[:, i]
        return U.copy(), V

    monkeypatch.setattr(og, "sign_fix", wrong)
    assert not _sign_pin()


def test_sign_fix_with_last_index_on_ties_is_caught(monkeypatch):
    def wrong(U, V):
        U, V = U.copy(), V.copy()
        for i in range(V.shape[1]):
            a = np.abs(V[:, i])
            idx = int(np.flatnonzero(a == a.max())[-1])
            if V[idx, i] < 0:
                V[:, i] = -V[:, i]
                U[:, i] = -U[:, i]
        return U, V

    monkeypatch.setattr(og, "sign_fix", wrong)
    assert not _sign_pin()


# ---------------------------------------------------------------------------
# principal angles: span{e1, e2} against span{e1, cos t e2 + sin t e3} = [0, t]
# ---------------------------------------------------------------------------

def _rotated_pair(theta, d=7, seed=0):
    E = np.eye(d)
    X = E[:, :2].copy()
    Y = np.stack([E[:, 0], np.cos(theta) * E[:, 1] + np.sin(theta) * E[:, 2]], axis=1)
    # hide the structure behind a random orthogonal change of coordinates and
    # random bases of both spans
    rng = np.random.default_rng(seed)
    Qr, _ = np.linalg.qr(rng.standard_normal((d, d)))
    Gx = rng.standard_normal((2, 2)) + 3 * np.eye(2)
    Gy = rng.standard_normal((2, 2)) + 3 * np.eye(2)
    return Qr @ X @ Gx, Qr @ Y @ Gy


def _angle_pin(theta):
    X, Y = _rotated_pair(theta)
    ang = og.subspace_angles(X, Y)
    return bool(ang.shape == (2,) and abs(ang[0]) <= 1e-15 + 1e-9 * theta
                and abs(ang[1] - theta) <= 1e-6 * theta + 1e-15)


@pytest.mark.parametrize("theta", [1.2, 0.3, 1e-3, 1e-5, 1e-7, 1e-9])
def test_subspace_angles_known_rotation(theta):
    assert _angle_pin(theta)


def test_subspace_angles_orthogonal_and_identical():
    E = np.eye(5)
    assert np.allclose(oracle.subspace_angles(E[:, :2], E[:, 2:4]), [np.pi / 2] * 2, atol=1e-15)
    X = np.random.default_rng(3).standard_normal((9, 3))
    assert np.max(oracle.subspace_angles(X, X @ np.diag([2.0, -1.0, 0.5]))) <= 1e-14


def test_subspace_angles_that_return_zeros_are_caught(monkeypatch):
    monkeypatch.setattr(og, "subspace_angles", lambda X, Y: np.zeros(X.shape[1]))
    assert not _angle_pin(1e-3)


def test_subspace_angles_by_arccos_alone_are_caught(monkeypatch):
    def wrong(X, Y):
        qx, _ = np.linalg.qr(X)
        qy, _ = np.linalg.qr(Y)
        c = np.linalg.svd(qx.T @ qy, compute_uv=False)
        return np.arccos(np.clip(c, -1.0, 1.0))[::-1]

    monkeypatch.setattr(og, "subspace_angles", wrong)
    # the zero angle comes out near 1e-8 and a 1e-9 angle is lost entirely
    assert not _angle_pin(1e-3)
    assert not _angle_pin(1e-9)


# ---------------------------------------------------------------------------
# residual certificate on an operator with a known SVD
# ---------------------------------------------------------------------------

def _known_svd(n=30, p=20, seed=1):
    rng = np.random.default_rng(seed)
    P, _ = np.linalg.qr(rng.standard_normal((n, p)))
    Q, _ = np.linalg.qr(rng.standard_normal((p, p)))
    s = np.linspace(10.0, 1.0, p)
    return og.DenseOperator(P @ np.diag(s) @ Q.T), s, P, Q


def _certificate_pin():
    op, s, P, Q = _known_svd()
    k = 4
    r1, r2, rq = og.certificate(op, s[:k], P[:, :k], Q[:, :k])
    exact_ok = max(r1.max(), r2.max()) <= 1e-13 * s[0] and np.allclose(rq, s[:k], rtol=1e-14)
    # sigma shifted by known deltas: both residuals equal |delta| (unit vectors)
    d = np.array([1e-3, -2e-6, 5e-9, 0.25])
    r1, r2, rq = og.certificate(op, s[:k] + d, P[:, :k], Q[:, :k])
    shift_ok = (np.allclose(r1, np.abs(d), rtol=1e-6, atol=1e-13)
                and np.allclose(r2, np.abs(d), rtol=1e-6, atol=1e-13)
                and np.allclose(rq, s[:k], rtol=1e-14))
    # right vector tilted by angle t towards q_{k+1}: ||A v - s u|| = sqrt((s cos t - s)^2
    # + (s_{k+1} sin t)^2), ||A^T u - s v|| = s sin t
    t = 1e-4
    V = Q[:, :k].copy()
    V[:, 0] = np.cos(t) * Q[:, 0] + np.sin(t) * Q[:, k]
    r1, r2, rq = og.certificate(op, s[:k], P[:, :k], V)
    want1 = np.hypot(s[0] * (np.cos(t) - 1.0), s[k] * np.sin(t))
    tilt_ok = (abs(r1[0] - want1) <= 1e-6 * want1 and abs(r2[0] - s[0] * np.sin(t)) <= 1e-6 * s[0] * t
               and abs(rq[0] - s[0] * np.cos(t)) <= 1e-13 * s[0])
    return bool(exact_ok and shift_ok and tilt_ok)


def test_certificate_known_residuals():
    assert _certificate_pin()


def test_certificate_bounds_sigma_error():
    # Weyl / residual bound: some exact singular value lies within max(r1, r2) of
    # each returned value
    op, s, P, Q = _known_svd(seed=4)
    d = 3e-4
    r1, r2, _ = og.certificate(op, s[:3] + d, P[:, :3], Q[:, :3])
    assert np.all(np.maximum(r1, r2) >= d * (1 - 1e-9))


def test_certificate_without_sigma_term_is_caught(monkeypatch):
    def wrong(op, sigma, U, V):
        k = len(sigma)
        r1, r2, rq = np.empty(k), np.empty(k), np.empty(k)
        for i in range(k):
            Av = op.matvec(V[:, i])
            Atu = op.rmatvec(U[:, i])
            r1[i] = np.linalg.norm(Av - U[:, i])          # sigma dropped
            r2[i] = np.linalg.norm(Atu - V[:, i])
            rq[i] = U[:, i] @ Av
        return r1, r2, rq

    monkeypatch.setattr(og, "certificate", wrong)
    assert not _certificate_pin()


def test_certificate_with_swapped_vectors_is_caught(monkeypatch):
    def wrong(op, sigma, U, V):
        k = len(sigma)
        r1, r2, rq = np.empty(k), np.empty(k), np.empty(k)
        for i in range(k):
            Av = op.matvec(V[:, i])
            Atu = op.rmatvec(U[:, i])
            r1[i] = np.linalg.norm(Av - sigma[i] * U[:, i])
            r2[i] = np.linalg.norm(Atu - sigma[i] * V[:, i])
            rq[i] = V[:, i] @ Atu if i == 0 else U[:, i] @ Av
            r2[i] = r1[i]                                  # one side reported twice
        return r1, r2, rq

    monkeypatch.setattr(og, "certificate", wrong)
    assert not _certificate_pin()
