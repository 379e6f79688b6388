"""GPU parity of the blocked GKL with FP64-accurate block products
(GKL_PREC_BLOCK_FP64: each column in seven int8 limbs of a 52-bit fixed point,
two columns per pass over the matrix).

Error model: every column is quantised exactly as the single-vector limb
products are (tests/test_gpu_limbs.py, tests/limb_bounds.py), with its own
power-of-two scale, and the limb sums are exact; per column the product is
within 1e-12 of its norm plus the quantisation slack, and it agrees with the
single-vector limb product to the rounding of the K-split sums.  The blocked
solve is FP64 everywhere else, so it is held to the FP64 targets: sigma within
1e-10 of the oracle, orthonormal bases, residual certificate <= 1e-9 sigma_1.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth   # noqa: E402
from limb_bounds import quantisation_slack  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_1808_03374_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


SHAPES = [("c1", 1000, 5000, None, 0), ("c2", 37, 513, 20, -1), ("c5", 1001, 333, None, -1),
          ("c2", 3000, 70000, None, -1)]


@pytest.mark.parametrize("b", [1, 2, 3, 5])
@pytest.mark.parametrize("name,n,p,ld,pad", SHAPES)
def test_block_fp64_products(gk, name, n, p, ld, pad, b):
    g = synth.config(name, n=n, p=p, ld=ld, pad_mode=pad)
    Gd = dev(g.packed)
    op = oracle.PackedOperator(g.packed, n, p)
    ctx = gk.Context(Gd, n, p, 1, precision=gk.GKL_PREC_BLOCK_FP64, block_width=2, krylov_dim=8)
    rng = np.random.default_rng(n + p + b)
    # columns of very different scales share a pass: each keeps its own scale
    scales = np.array([1.0, 1e-100, 1e100, 3.0, 1e-3])[:b]
    W = rng.standard_normal((p, b)) * scales
    X = rng.standard_normal((n, b)) * scales
    Y = ctx.matmat_mixed(dev(W)).cpu().numpy()
    Z = ctx.rmatmat_mixed(dev(X)).cpu().numpy()
    ctx.close()
    for c in range(b):
        y0, z0 = op.matvec(W[:, c]), op.rmatvec(X[:, c])
        sy, sz = quantisation_slack(g, W[:, c], X[:, c])
        assert np.linalg.norm(Y[:, c] - y0) <= 1e-12 * np.linalg.norm(y0) + sy, c
        assert np.linalg.norm(Z[:, c] - z0) <= 1e-12 * np.linalg.norm(z0) + sz, c


def test_block_fp64_pairs_match_single_vector_limbs(gk):
    # the same integer limb sums: the pair pass and the single-vector limb
    # product differ only in the order the K-split partials are added
    g = synth.config("c2", n=4000, p=50000)
    Gd = dev(g.packed)
    rng = np.random.default_rng(17)
    W = rng.standard_normal((g.p, 2))
    X = rng.standard_normal((g.n, 2))
    blk = gk.Context(Gd, g.n, g.p, 1, precision=gk.GKL_PREC_BLOCK_FP64, block_width=2, krylov_dim=8)
    Y = blk.matmat_mixed(dev(W)).cpu().numpy()
    Z = blk.rmatmat_mixed(dev(X)).cpu().numpy()
    blk.close()
    one = gk.Context(Gd, g.n, g.p, 1, fp64_products=gk.GKL_FP64_LIMBS)
    for c in range(2):
        y1 = one.matvec(dev(W[:, c])).cpu().numpy()
        z1 = one.rmatvec(dev(X[:, c])).cpu().numpy()
        assert np.linalg.norm(Y[:, c] - y1) <= 1e-14 * np.linalg.norm(y1)
        assert np.linalg.norm(Z[:, c] - z1) <= 1e-14 * np.linalg.norm(z1)
    one.close()


def test_block_fp64_products_full_size_sampled(gk):
    # the full 10,000 x 100,000 workload, one pair, sampled rows and SNPs
    g = synth.config("c2")
    n, p = g.n, g.p
    op = oracle.PackedOperator(g.packed, n, p)
    ctx = gk.Context(dev(g.packed), n, p, 1, precision=gk.GKL_PREC_BLOCK_FP64, block_width=2,
                     krylov_dim=8)
    rng = np.random.default_rng(5)
    W = rng.standard_normal((p, 2))
    X = rng.standard_normal((n, 2))
    Y = ctx.matmat_mixed(dev(W)).cpu().numpy()
    Z = ctx.rmatmat_mixed(dev(X)).cpu().numpy()
    ctx.close()
    rows = np.concatenate([[0, n - 1], rng.choice(n, 30, replace=False)])
    cols = np.concatenate([[0, p - 1], rng.choice(p, 30, replace=False)])
    for c in range(2):
        assert np.max(np.abs(Y[rows, c] - op.matvec_rows(W[:, c], rows))) <= \
            1e-12 * np.linalg.norm(Y[:, c]) / np.sqrt(n) * 10
        assert np.max(np.abs(Z[cols, c] - op.rmatvec_cols(X[:, c], cols))) <= \
            1e-12 * np.linalg.norm(Z[:, c]) / np.sqrt(p) * 10


@pytest.mark.parametrize("b,m", [(1, 0), (2, 0), (3, 0), (4, 0), (2, 48), (3, 48)])
def test_block_fp64_solve_matches_oracle(gk, b, m):
    g = synth.config("c2", n=2000, p=20000)
    k = 20
    op = oracle.PackedOperator(g.packed, g.n, g.p)
    ref = oracle.gkl_svd(op, k, tol=1e-12, v0=synth.start_vector(g.p, 3),
                         spare_left=synth.spare_directions(g.n, 8, 3),
                         spare_right=synth.spare_directions(g.p, 8, 3))
    extra = {"krylov_dim": m} if m else {}
    ctx = gk.Context(dev(g.packed), g.n, g.p, k, tol=1e-11, precision=gk.GKL_PREC_BLOCK_FP64,
                     block_width=b, **extra)
    sigma, U, V, st, info = ctx.solve()
    assert st == gk.GKL_OK, gk.gkl_last_error(ctx.ctx)
    ctx.close()
    sigma = sigma.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    assert np.all(np.abs(sigma - ref.sigma) <= 1e-10 * ref.sigma)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-10
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-10
    r1, r2, _ = oracle.certificate(op, sigma, U, V)
    assert max(r1.max(), r2.max()) <= 1e-9 * sigma[0]
    # one pass over the matrix per pair of columns
    assert info.passes_over_G * b == info.matvecs * ((b + 1) // 2)
    if m:
        assert info.restarts > 0


def test_block_fp64_not_for_loco(gk):
    # LOCO's shared width-22 block products keep the matrix-core formats
    rng = np.random.default_rng(2)
    packed = rng.integers(0, 256, size=(900, 100), dtype=np.uint8)
    with pytest.raises(gk.GKLError):
        gk.LocoContext(dev(packed), 400, 900, [0, 500, 900], 3, precision=gk.GKL_PREC_BLOCK_FP64)


def _dense_sigma(packed, n, p, k):
    st = oracle.column_stats(n, *oracle.counts(packed, n, p))
    A = oracle.dense_matrix(oracle.decode(packed, n, p), st.mean, st.inv_sd)
    return np.linalg.svd(A, compute_uv=False)[:k]


@pytest.mark.parametrize("fmt,tol_sigma", [("BLOCK_FP64", 1e-10), ("MIXED", 1e-6), ("MIXED_INT8", 1e-6)])
@pytest.mark.parametrize("b", [2, 3])
def test_small_blocks_on_rank_deficient_matrices(gk, fmt, tol_sigma, b):
    # blocks of 2 and 3 columns (the row-parallel block QR and the fused block
    # Gram-Schmidt) on a matrix of rank at most 8: the Krylov space runs out and
    # the blocks turn dependent, so the shifted Cholesky QR and the breakdown
    # handling are exercised; the top singular values still come out right
    rng = np.random.default_rng(40 + b)
    n, p, r = 400, 1200, 8
    base = rng.integers(0, 3, size=(n, r))
    codes = base[:, rng.integers(0, r, size=p)]
    packed = synth.pack_codes(codes)
    k = 4
    ref = _dense_sigma(packed, n, p, k)
    # the budget bounds the run if the breakdown handling ever fails
    ctx = gk.Context(dev(packed), n, p, k, tol=1e-11, precision=getattr(gk, "GKL_PREC_" + fmt),
                     block_width=b, krylov_dim=24, max_matvecs=3000)
    sigma, U, V, st, info = ctx.solve()
    ctx.close()
    assert st == gk.GKL_OK, (st, info.matvecs, info.restarts)
    sigma = sigma.cpu().numpy()
    assert np.all(np.abs(sigma - ref) <= tol_sigma * ref[0]), (sigma, ref)
    V = V.cpu().numpy()
    U = U.cpu().numpy()
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-8
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-8
