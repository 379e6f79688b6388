"""ORACLE -- test infrastructure only (see the package docstring).

Plain FP64 Golub-Kahan-Lanczos bidiagonalisation with full reorthogonalisation
by doubly reorthogonalised classical Gram-Schmidt (CGS2), no restart, on the
implicitly standardised genotype matrix.

Paper passages followed:
  * Section 3 (GKL bidiagonalisation, Golub & Kahan 1965): A V_j = U_j B_j with
    B_j upper bidiagonal; the top singular triplets come from the SVD of B_j.
  * Section 3, "Choice of reorthogonalization strategy": full reorthogonalisation
    with doubly reorthogonalised classical Gram-Schmidt.  The oracle always runs
    both passes.
  * Section 3, "Convergence criteria" and the Table 3 caption: the residual bound
    |sigma - sigma~_i| <= beta_j |P_{j,i}| (last row of the left singular vectors
    of B_j); the sum of these over the top k is the paper's ||Delta theta||_1.
  * Section 4 (ARPACK paragraph): the eigenvalues of [0 X; X^T 0] are +-sigma,
    used as a pin in the tests.
  * Section 2, eq. (mplaw-ev) and (mplaw-sv): Marchenko-Pastur densities, read
    with denominator 2 pi sigma^2 min(1, rho) xi (eigenvalues) and
    pi sigma^2 min(1, rho) x (singular values), rho = rows / columns.

  * Section 3, "Thick restarting": restarts that keep l Ritz vectors, from
    ordinary Ritz values (Wu & Simon 2000) or from harmonic Ritz values (Baglama
    & Reichel, SIAM J. Sci. Comput. 27, 2005).  Here the harmonic Ritz pairs
    are those of A^T A on span(V_m) with the Petrov condition taken against
    A^T A V_m; their values are the squared singular values of [B_m, beta_m e_m]
    and their vectors V_m B_m^-1 p_j (p_j its left singular vectors), formed
    from the right singular vectors and the null vector of [B_m, beta_m e_m].

Readings where the paper is silent (listed with the rest in the design notes):
  * preprocessing: column centring by the observed mean and scaling by
    1/sqrt(2 f (1 - f)), f = mean / 2; missing entries mean-imputed (zero);
    s = 0 for monomorphic or fully missing columns;
  * start vector: a seeded Gaussian, normalised; breakdown (alpha or beta below
    eps * ||B|| * sqrt(max(n, p))) continues with a supplied random direction
    orthogonalised against the basis and records a zero scalar;
  * sign rule: the largest-magnitude entry of each right singular vector is
    positive (lowest index on ties); the left vector flips with it.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build_library(force: bool = False) -> str:
    """Compile packed.c (plain C99 + OpenMP, no FP contraction) into liboracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-ffp-contract=off", os.path.join(_HERE, "packed.c"), "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build_library()
            lib = ctypes.CDLL(_LIB_PATH)
            i64, vp = ctypes.c_int64, ctypes.c_void_p
            lib.oracle_decode.argtypes = [vp, i64, i64, i64, vp]
            lib.oracle_counts.argtypes = [vp, i64, i64, i64, vp, vp, vp]
            lib.oracle_matvec.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp]
            lib.oracle_rmatvec.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp]
            lib.oracle_matvec_rows.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, i64, vp]
            lib.oracle_rmatvec_cols.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, i64, vp]
            for f in (lib.oracle_decode, lib.oracle_counts, lib.oracle_matvec,
                      lib.oracle_rmatvec, lib.oracle_matvec_rows, lib.oracle_rmatvec_cols):
                f.restype = None
            _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _check_packed(packed, n, p):
    packed = np.ascontiguousarray(packed, dtype=np.uint8)
    if packed.ndim != 2 or packed.shape[0] != p or packed.shape[1] < (n + 3) // 4:
        raise ValueError("packed must have shape (p, ld) with ld >= ceil(n/4)")
    return packed, packed.shape[1]


# ---------------------------------------------------------------------------
# Decode and column statistics
# ---------------------------------------------------------------------------

def decode(packed: np.ndarray, n: int, p: int) -> np.ndarray:
    """(n, p) int8 matrix of genotypes 0/1/2, -1 for missing (storage-format reading)."""
    packed, ld = _check_packed(packed, n, p)
    out = np.empty((p, n), dtype=np.int8)
    _load().oracle_decode(_p(packed), n, p, ld, _p(out))
    return out.T


def counts(packed: np.ndarray, n: int, p: int):
    """Per-SNP counts (n1, n2, n3) of codes 1, 2 and missing."""
    packed, ld = _check_packed(packed, n, p)
    n1 = np.empty(p, dtype=np.int64)
    n2 = np.empty(p, dtype=np.int64)
    n3 = np.empty(p, dtype=np.int64)
    _load().oracle_counts(_p(packed), n, p, ld, _p(n1), _p(n2), _p(n3))
    return n1, n2, n3


@dataclasses.dataclass
class ColumnStats:
    n1: np.ndarray
    n2: np.ndarray
    n3: np.ndarray
    count: np.ndarray     # allele count c = n1 + 2 n2 (int64)
    nobs: np.ndarray      # observed individuals n - n3 (int64)
    mean: np.ndarray      # mu = c / nobs
    inv_sd: np.ndarray    # s = 1 / sqrt(mu (1 - mu/2)), 0 when undefined


def column_stats(n: int, n1: np.ndarray, n2: np.ndarray, n3: np.ndarray) -> ColumnStats:
    """Column centring and scaling from exact integer counts.

    Fixed IEEE operation order, one correctly rounded operation per step:
    mu = c / nobs; f = 0.5 mu; t = 1 - f; var = mu t; d = sqrt(var); s = 1 / d.
    """
    n1 = np.asarray(n1, dtype=np.int64)
    n2 = np.asarray(n2, dtype=np.int64)
    n3 = np.asarray(n3, dtype=np.int64)
    nobs = np.int64(n) - n3
    c = n1 + 2 * n2
    mean = np.zeros(nobs.shape, dtype=np.float64)
    inv_sd = np.zeros(nobs.shape, dtype=np.float64)
    ok = nobs > 0
    mu = c[ok].astype(np.float64) / nobs[ok].astype(np.float64)
    f = 0.5 * mu
    t = 1.0 - f
    var = mu * t
    d = np.sqrt(var)
    with np.errstate(divide="ignore"):
        s = np.where(var > 0.0, 1.0 / np.where(var > 0.0, d, 1.0), 0.0)
    mean[ok] = mu
    inv_sd[ok] = s
    return ColumnStats(n1, n2, n3, c, nobs, mean, inv_sd)


def dense_matrix(codes: np.ndarray, mean: np.ndarray, inv_sd: np.ndarray) -> np.ndarray:
    """Explicit standardised A (n x p FP64): A_ij = o_ij (g_ij - mu_j) s_j."""
    g = codes.astype(np.float64)
    obs = codes >= 0
    return np.where(obs, (g - mean[None, :]) * inv_sd[None, :], 0.0)


def frobenius_sq_from_counts(st: ColumnStats) -> float:
    """||A||_F^2 = sum_j s_j^2 (sum_i g_ij^2 - c_j^2 / nobs_j), from integer counts."""
    sumsq = (st.n1 + 4 * st.n2).astype(np.float64)
    ok = st.nobs > 0
    cen = np.zeros_like(sumsq)
    cen[ok] = sumsq[ok] - st.count[ok].astype(np.float64) ** 2 / st.nobs[ok]
    return float(np.sum(st.inv_sd ** 2 * cen))


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------

class DenseOperator:
    """A held explicitly (small sizes)."""

    def __init__(self, A: np.ndarray):
        self.A = np.asarray(A, dtype=np.float64)
        self.shape = self.A.shape
        self.matvecs = 0

    def matvec(self, v):
        self.matvecs += 1
        return self.A @ v

    def rmatvec(self, u):
        self.matvecs += 1
        return self.A.T @ u


class PackedOperator:
    """A applied from the packed bytes by the plain C loops in packed.c."""

    def __init__(self, packed: np.ndarray, n: int, p: int, stats: ColumnStats | None = None):
        self.packed, self.ld = _check_packed(packed, n, p)
        self.n, self.p = n, p
        self.shape = (n, p)
        if stats is None:
            stats = column_stats(n, *counts(self.packed, n, p))
        self.stats = stats
        self.mean = np.ascontiguousarray(stats.mean)
        self.inv_sd = np.ascontiguousarray(stats.inv_sd)
        self.matvecs = 0

    def matvec(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        y = np.empty(self.n)
        _load().oracle_matvec(_p(self.packed), self.n, self.p, self.ld, _p(self.mean),
                              _p(self.inv_sd), _p(v), _p(y))
        self.matvecs += 1
        return y

    def rmatvec(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        z = np.empty(self.p)
        _load().oracle_rmatvec(_p(self.packed), self.n, self.p, self.ld, _p(self.mean),
                               _p(self.inv_sd), _p(u), _p(z))
        self.matvecs += 1
        return z

    def matvec_rows(self, v, rows):
        v = np.ascontiguousarray(v, dtype=np.float64)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        y = np.empty(rows.size)
        _load().oracle_matvec_rows(_p(self.packed), self.n, self.p, self.ld, _p(self.mean),
                                   _p(self.inv_sd), _p(v), _p(rows), rows.size, _p(y))
        return y

    def rmatvec_cols(self, u, cols):
        u = np.ascontiguousarray(u, dtype=np.float64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        z = np.empty(cols.size)
        _load().oracle_rmatvec_cols(_p(self.packed), self.n, self.p, self.ld, _p(self.mean),
                                    _p(self.inv_sd), _p(u), _p(cols), cols.size, _p(z))
        return z


# ---------------------------------------------------------------------------
# GKL with full CGS2 reorthogonalisation, no restart
# ---------------------------------------------------------------------------

def cgs2(Q: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Classical Gram-Schmidt run twice: r <- r - Q (Q^T r), both passes always."""
    if Q.shape[1] == 0:
        return r
    r = r - Q @ (Q.T @ r)
    r = r - Q @ (Q.T @ r)
    return r


@dataclasses.dataclass
class GKLResult:
    sigma: np.ndarray          # k, descending
    U: np.ndarray              # n x k
    V: np.ndarray              # p x k
    residuals: np.ndarray      # k, beta_j |P_{j,i}|
    alphas: np.ndarray         # steps
    betas: np.ndarray          # steps
    steps: int
    matvecs: int
    converged: bool
    breakdowns: int


def sign_fix(U: np.ndarray, V: np.ndarray):
    """Make the largest-|.| entry of each column of V positive (first index on ties)."""
    U = U.copy()
    V = V.copy()
    for i in range(V.shape[1]):
        idx = int(np.argmax(np.abs(V[:, i])))
        if V[idx, i] < 0:
            V[:, i] = -V[:, i]
            U[:, i] = -U[:, i]
    return U, V


def _bidiag(alphas, betas):
    m = len(alphas)
    B = np.diag(np.asarray(alphas, dtype=np.float64))
    if m > 1:
        B += np.diag(np.asarray(betas[: m - 1], dtype=np.float64), 1)
    return B


def gkl_svd(op, k: int, tol: float = 1e-12, v0: np.ndarray | None = None,
            max_steps: int | None = None, spare_left: np.ndarray | None = None,
            spare_right: np.ndarray | None = None, check_every: int = 1) -> GKLResult:
    """Top-k singular triplets of the operator by plain GKL (see module docstring).

    Steps j = 1, 2, ...:
        p  = A v_j - beta_{j-1} u_{j-1};  CGS2 against u_1..u_{j-1};
        alpha_j = ||p||;  u_j = p / alpha_j
        r  = A^T u_j - alpha_j v_j;       CGS2 against v_1..v_j;
        beta_j = ||r||;   v_{j+1} = r / beta_j
    B_j = bidiag(alpha, beta);  B_j = P S Q^T;  residual_i = beta_j |P[j, i]|.
    Stops when residual_i <= tol * S[0] for every i < k, or at min(n, p) steps.
    """
    n, p = op.shape
    if not (1 <= k <= min(n, p)):
        raise ValueError("k must lie in [1, min(n, p)]")
    mmax = min(n, p) if max_steps is None else min(int(max_steps), min(n, p))
    if v0 is None:
        v0 = np.random.default_rng(0).standard_normal(p)
    eps = np.finfo(np.float64).eps
    U = np.zeros((n, mmax))
    V = np.zeros((p, mmax + 1))
    alphas = np.zeros(mmax)
    betas = np.zeros(mmax)
    V[:, 0] = v0 / np.linalg.norm(v0)
    norm_est = 0.0
    nl = nr = 0
    breakdowns = 0
    start_mv = op.matvecs
    converged = False
    P = S = Qt = None
    j = -1
    for j in range(mmax):
        w = op.matvec(V[:, j])
        if j > 0:
            w = w - betas[j - 1] * U[:, j - 1]
        w = cgs2(U[:, :j], w)
        a = float(np.linalg.norm(w))
        norm_est = max(norm_est, a)
        if a <= eps * norm_est * np.sqrt(max(n, p)):
            breakdowns += 1
            a = 0.0
            if spare_left is None or nl >= spare_left.shape[0]:
                raise RuntimeError("breakdown on the left side and no spare direction left")
            w = cgs2(U[:, :j], spare_left[nl].astype(np.float64))
            nl += 1
            w = w / np.linalg.norm(w)
            U[:, j] = w
        else:
            U[:, j] = w / a
        alphas[j] = a
        r = op.rmatvec(U[:, j]) - a * V[:, j]
        r = cgs2(V[:, : j + 1], r)
        b = float(np.linalg.norm(r))
        norm_est = max(norm_est, np.hypot(a, b))
        if b <= eps * norm_est * np.sqrt(max(n, p)):
            breakdowns += 1
            b = 0.0
            if j + 1 < min(n, p) and j + 1 < mmax:
                if spare_right is None or nr >= spare_right.shape[0]:
                    raise RuntimeError("breakdown on the right side and no spare direction left")
                r = cgs2(V[:, : j + 1], spare_right[nr].astype(np.float64))
                nr += 1
                V[:, j + 1] = r / np.linalg.norm(r)
        else:
            V[:, j + 1] = r / b
        betas[j] = b
        steps = j + 1
        if steps >= k and (steps % check_every == 0 or steps == mmax):
            P, S, Qt = np.linalg.svd(_bidiag(alphas[:steps], betas[:steps]))
            res = b * np.abs(P[j, :])
            if np.all(res[:k] <= tol * S[0]):
                converged = True
                break
    steps = j + 1
    if P is None or P.shape[0] != steps:
        P, S, Qt = np.linalg.svd(_bidiag(alphas[:steps], betas[:steps]))
    res = betas[steps - 1] * np.abs(P[steps - 1, :])
    Uk = U[:, :steps] @ P[:, :k]
    Vk = V[:, :steps] @ Qt.T[:, :k]
    Uk, Vk = sign_fix(Uk, Vk)
    return GKLResult(S[:k].copy(), Uk, Vk, res[:k].copy(), alphas[:steps].copy(),
                     betas[:steps].copy(), steps, op.matvecs - start_mv, converged, breakdowns)


# ---------------------------------------------------------------------------
# Thick restart (ordinary or harmonic Ritz vectors), full CGS2
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class RestartPlan:
    Yl: np.ndarray       # m x l: new left basis U_m Yl
    Z: np.ndarray        # (m+1) x (l+1): new right basis V_{m+1} Z
    H: np.ndarray        # l x l: U_new^T A V_new[:, :l]
    c: np.ndarray        # l: U_new^T A V_new[:, l]
    values: np.ndarray   # l: the Ritz (or harmonic Ritz) singular values kept


def thick_restart(B: np.ndarray, beta_m: float, l: int, kind: str) -> RestartPlan:
    """Small-space part of a thick restart after m steps (Section 3, "Thick
    restarting"), from A V_m = U_m B and A^T U_m = V_m B^T + beta_m v_{m+1} e_m^T.

    kind "ritz" (Wu & Simon): B = P S Q^T; keep U_m P_l, V_m Q_l and v_{m+1}.
    kind "harmonic" (Baglama & Reichel): with [B, beta_m e_m] = Ph Sh Qh^T, the
    harmonic Ritz vectors are V_m B^-1 Ph_l and their residuals all lie along
    V_{m+1} w, w = [-beta_m B^-1 e_m; 1].  Since [B, beta_m e_m] w = 0, w spans
    the null space of [B, beta_m e_m] (its last right singular vector), and
    sigma_j [B^-1 ph_j; 0] = qh_j - qh_j(m+1) w, so the kept space is
    span{qh_1..qh_l, w} and the harmonic vectors are its members with a zero
    last coordinate.  Both come from the SVD without B^-1, which is nearly
    singular when the Krylov space holds a near-null vector of A (a wide
    genotype matrix).  One Householder reflection of [qh_1..qh_l, w] zeroes the
    last coordinate of its first l columns; the left vectors are U_m Ph_l.
    H and c follow from their definitions through A V_m = U_m B and
    u^T A v_{m+1} = (A^T u)^T v_{m+1} = beta_m (e_m^T y) for u = U_m y.
    """
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
    elif kind == "harmonic":
        Bh = np.hstack([B, beta_m * em[:, None]])
        Ph, Sh, Qht = np.linalg.svd(Bh, full_matrices=True)
        Yl = Ph[:, :l]
        QS = np.hstack([Qht[:l].T, Qht[m][:, None]])
        r = QS[m, :]
        v = r.copy()
        v[l] += np.copysign(np.linalg.norm(r), r[l])
        Z = QS - np.outer(QS @ v, (2.0 / (v @ v)) * v)
        Z[m, :l] = 0.0
        values = Sh[:l].copy()
    else:
        raise ValueError("kind must be 'ritz' or 'harmonic'")
    H = Yl.T @ B @ Z[:m, :l]
    c = Yl.T @ B @ Z[:m, l] + Z[m, l] * beta_m * Yl[m - 1, :]
    return RestartPlan(Yl, Z, H, c, values)


def gkl_svd_thick(op, k: int, tol: float, krylov: int, keep: int, restart: str = "ritz",
                  v0: np.ndarray | None = None, max_restarts: int = 1000) -> GKLResult:
    """Top-k singular triplets by GKL with full CGS2 and thick restarts.

    The basis grows to m = krylov vectors; then the residual test of gkl_svd
    runs on the projected matrix B (its first l rows hold the restart head H and
    the coupling column c after a restart, the rest is bidiagonal), and if it
    fails, thick_restart keeps l = keep vectors.  The first step after a restart
    subtracts U_l c from A v_l (the coupling), every other step beta u_{j-1}.
    alphas and betas list every step, across restarts.
    """
    n, p = op.shape
    m = int(krylov)
    if not (1 <= k <= keep < m <= min(n, p)):
        raise ValueError("need 1 <= k <= keep < krylov <= min(n, p)")
    if v0 is None:
        v0 = np.random.default_rng(0).standard_normal(p)
    U = np.zeros((n, m))
    V = np.zeros((p, m + 1))
    B = np.zeros((m, m))
    V[:, 0] = v0 / np.linalg.norm(v0)
    alphas, betas = [], []
    start_mv = op.matvecs
    nlock = 0
    restarts = 0
    j = 0
    converged = False
    while True:
        w = op.matvec(V[:, j])
        if j > 0 and j == nlock:
            w = w - U[:, :nlock] @ B[:nlock, nlock]
        elif j > 0:
            w = w - B[j - 1, j] * U[:, j - 1]
        w = cgs2(U[:, :j], w)
        a = float(np.linalg.norm(w))
        U[:, j] = w / a
        B[j, j] = a
        r = op.rmatvec(U[:, j]) - a * V[:, j]
        r = cgs2(V[:, : j + 1], r)
        b = float(np.linalg.norm(r))
        V[:, j + 1] = r / b
        if j + 1 < m:
            B[j, j + 1] = b
        alphas.append(a)
        betas.append(b)
        j += 1
        if j < m:
            continue
        P, S, Qt = np.linalg.svd(B)
        res = b * np.abs(P[m - 1, :])
        if np.all(res[:k] <= tol * S[0]):
            converged = True
            break
        if restarts >= max_restarts:
            break
        plan = thick_restart(B, b, keep, restart)
        U[:, :keep] = U @ plan.Yl
        V[:, : keep + 1] = V @ plan.Z
        B = np.zeros((m, m))
        B[:keep, :keep] = plan.H
        B[:keep, keep] = plan.c
        nlock = keep
        j = keep
        restarts += 1
    Uk = U @ P[:, :k]
    Vk = V[:, :m] @ Qt.T[:, :k]
    Uk, Vk = sign_fix(Uk, Vk)
    out = GKLResult(S[:k].copy(), Uk, Vk, res[:k].copy(), np.array(alphas), np.array(betas),
                    len(alphas), op.matvecs - start_mv, converged, 0)
    out.restarts = restarts
    return out


def certificate(op, sigma, U, V):
    """Residual norms ||A v_i - sigma_i u_i||, ||A^T u_i - sigma_i v_i|| and the
    Rayleigh quotients u_i^T A v_i; each residual bounds |sigma_i - sigma_true|."""
    k = len(sigma)
    r1 = np.empty(k)
    r2 = np.empty(k)
    rq = np.empty(k)
    for i in range(k):
        Av = op.matvec(V[:, i])
        Atu = op.rmatvec(U[:, i])
        r1[i] = np.linalg.norm(Av - sigma[i] * U[:, i])
        r2[i] = np.linalg.norm(Atu - sigma[i] * V[:, i])
        rq[i] = U[:, i] @ Av
    return r1, r2, rq


def subspace_angles(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Principal angles (radians, ascending) between the column spaces of X and Y
    (same number of columns).

    The cosines are the singular values of Qx^T Qy and the sines those of the
    part of Qy outside span(Qx), Qy - Qx (Qx^T Qy) (Bjorck & Golub, Math. Comp.
    1973).  The i-th smallest angle pairs the i-th largest cosine with the i-th
    smallest sine; atan2 of the pair is accurate for every angle, where arccos of
    the cosine alone cannot resolve angles below about 1e-8.
    """
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    if qx.shape[1] != qy.shape[1]:
        raise ValueError("subspace_angles needs subspaces of equal dimension")
    M = qx.T @ qy
    c = np.linalg.svd(M, compute_uv=False)                    # descending
    s = np.linalg.svd(qy - qx @ M, compute_uv=False)[::-1]    # ascending
    return np.arctan2(np.clip(s, 0.0, 1.0), np.clip(c, 0.0, 1.0))


# ---------------------------------------------------------------------------
# Marchenko-Pastur law (eq. mplaw-ev, mplaw-sv)
# ---------------------------------------------------------------------------

def mp_singular_edges(rho: float, sigma: float = 1.0):
    """(sigma_-, sigma_+) = sigma |1 -+ sqrt(rho)|."""
    return sigma * abs(1.0 - np.sqrt(rho)), sigma * (1.0 + np.sqrt(rho))


def mp_eigen_density(xi, rho: float, sigma: float = 1.0):
    """Density of the non-zero eigenvalues: sqrt((l+ - xi)(xi - l-)) / (2 pi s^2 min(1, rho) xi)."""
    xi = np.asarray(xi, dtype=np.float64)
    lm = sigma ** 2 * (1.0 - np.sqrt(rho)) ** 2
    lp = sigma ** 2 * (1.0 + np.sqrt(rho)) ** 2
    inside = (xi > lm) & (xi < lp)
    out = np.zeros_like(xi)
    x = xi[inside]
    out[inside] = np.sqrt((lp - x) * (x - lm)) / (2.0 * np.pi * sigma ** 2 * min(1.0, rho) * x)
    return out


def mp_singular_density(x, rho: float, sigma: float = 1.0):
    """Density of the singular values: sqrt((s+^2 - x^2)(x^2 - s-^2)) / (pi s^2 min(1, rho) x)."""
    x = np.asarray(x, dtype=np.float64)
    sm, sp = mp_singular_edges(rho, sigma)
    inside = (x > sm) & (x < sp)
    out = np.zeros_like(x)
    y = x[inside]
    out[inside] = np.sqrt((sp ** 2 - y ** 2) * (y ** 2 - sm ** 2)) / (
        np.pi * sigma ** 2 * min(1.0, rho) * y)
    return out
