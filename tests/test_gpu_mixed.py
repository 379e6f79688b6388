"""GPU parity of the blocked mixed-precision path, with both matrix-core formats
of its products: split-BF16 vector tiles (GKL_PREC_MIXED) and exact int8 limbs
(GKL_PREC_MIXED_INT8).

Error model and tolerances
  * Int8 limbs: each vector column is rounded to integers of 22 bits below a
    power-of-two scale under twice its largest entry (three times that for the
    missing-term vector, which shares the scale), accumulation is exact, so per
    element the product error is at most 3 * 2^-22 max|w| times the row's sum of
    |codes| -- inside the split-BF16 bound below for vectors whose entries are
    within a factor of ten of their maximum, as random and Lanczos vectors are.
  * Split BF16: the vector block is split into bf16 hi + lo: |w - hi - lo| <= 2^-16 |w| per
    element; genotype operands are exact.  FP32 accumulation runs over chunks of
    1,024 K values (error ~ sqrt(4096) * 2^-24 of the chunk magnitude, about 4e-6
    relative to |A| |w|) and FP64 across chunks.  Per output element the error is
    therefore bounded by about 2^-16 (|A| |W|)_ic + 4e-6 (|A| |W|)_ic; the test
    uses 3e-5 (|A| |W|)_ic.
  * Singular values of the blocked solve agree with the FP64 oracle to 1e-6
    relative (the target for the mixed path).
  * Vectors (gap rule): a computed triplet's residual against the exact
    operator is at most eps * sigma_1, eps = solve tolerance + the measured
    error of the block products (the larger of ||dY|| / (sigma_1 ||w||) for
    A W and ||dZ|| / (sigma_1 ||x||) for A^T X on random unit vectors), so a
    singular vector with relative gap delta_i is within sin(angle) <= eps
    sigma_1 / (delta_i sigma_i) of the oracle's (Wedin's bound).  Every left and right vector whose
    bound is at most 1e-6 must be within 1e-6 rad; every other vector whose
    bound is below 0.1 must be within 10 times its bound.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth   # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_1808_03374_amd as m
    return m


PRECISIONS = ["bf16", "int8"]


def prec(gk, name):
    return gk.GKL_PREC_MIXED if name == "bf16" else gk.GKL_PREC_MIXED_INT8


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _dense(g):
    st = oracle.column_stats(g.n, *oracle.counts(g.packed, g.n, g.p))
    return oracle.dense_matrix(oracle.decode(g.packed, g.n, g.p), st.mean, st.inv_sd)


@pytest.mark.parametrize("fmt", PRECISIONS)
@pytest.mark.parametrize("name,n,p,b,pad", [("c1", 300, 900, 16, 0), ("c3", 523, 1111, 7, -1),
                                            ("c5", 1000, 3000, 32, -1), ("c2", 17, 260, 1, -1)])
def test_mixed_products(gk, name, n, p, b, pad, fmt):
    g = synth.config(name, n=n, p=p, pad_mode=pad)
    A = _dense(g)
    bw = 16 if min(n, p) >= 32 else 4
    ctx = gk.Context(dev(g.packed), n, p, 1, precision=prec(gk, fmt), block_width=bw,
                     krylov_dim=2 * bw)
    rng = np.random.default_rng(n + p + b)
    W = rng.standard_normal((p, b))
    X = rng.standard_normal((n, b))
    Y = ctx.matmat_mixed(dev(W)).cpu().numpy()
    Z = ctx.rmatmat_mixed(dev(X)).cpu().numpy()
    Y0 = A @ W
    Z0 = A.T @ X
    bound_y = 3e-5 * (np.abs(A) @ np.abs(W))
    bound_z = 3e-5 * (np.abs(A).T @ np.abs(X))
    assert np.all(np.abs(Y - Y0) <= bound_y + 1e-12)
    assert np.all(np.abs(Z - Z0) <= bound_z + 1e-12)
    # the error is far below the bound on average (random rounding)
    assert np.linalg.norm(Y - Y0) <= 1e-5 * np.linalg.norm(Y0)
    ctx.close()


def _oracle(g, k):
    op = oracle.PackedOperator(g.packed, g.n, g.p)
    return op, oracle.gkl_svd(op, k, tol=1e-12, v0=synth.start_vector(g.p, 3))


# m: basis size (None: the default); 120 and 128 take the projected SVD whose
# rotations are logged and replayed (more than 96 columns)
@pytest.mark.parametrize("name,n,p,k,b,m", [("c1", 1000, 5000, 10, 16, None),
                                            ("c3", 2000, 20000, 20, 16, None),
                                            ("c2", 2000, 20000, 20, 32, None),
                                            ("c3", 3000, 30000, 20, 8, None),
                                            ("c1", 1000, 5000, 10, 5, None),
                                            ("c3", 3000, 30000, 20, 8, 128),
                                            ("c1", 1000, 5000, 10, 5, 120)])
@pytest.mark.parametrize("fmt", PRECISIONS)
def test_mixed_solve_matches_fp64_oracle(gk, name, n, p, k, b, m, fmt):
    g = synth.config(name, n=n, p=p)
    op, ref = _oracle(g, k)
    extra = {} if m is None else {"krylov_dim": m}
    ctx = gk.Context(dev(g.packed), g.n, g.p, k, tol=1e-9, precision=prec(gk, fmt),
                     block_width=b, **extra)
    sigma, U, V, st, info = ctx.solve()
    assert st == gk.GKL_OK, gk.gkl_last_error(ctx.ctx)
    sigma = sigma.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    rel = np.abs(sigma - ref.sigma) / ref.sigma
    assert rel.max() <= 1e-6, rel
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-8
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-8
    # gap rule with the measured product error
    rng = np.random.default_rng(99)
    Wp = rng.standard_normal((g.p, 4))
    Wp /= np.linalg.norm(Wp, axis=0)
    Xp = rng.standard_normal((g.n, 4))
    Xp /= np.linalg.norm(Xp, axis=0)
    Ym = ctx.matmat_mixed(dev(Wp)).cpu().numpy()
    Zm = ctx.rmatmat_mixed(dev(Xp)).cpu().numpy()
    ctx.close()
    Y0 = np.stack([op.matvec(Wp[:, c]) for c in range(4)], axis=1)
    Z0 = np.stack([op.rmatvec(Xp[:, c]) for c in range(4)], axis=1)
    eps = 1e-9 + max(np.linalg.norm(Ym - Y0, axis=0).max(),
                     np.linalg.norm(Zm - Z0, axis=0).max()) / ref.sigma[0]
    gaps = np.abs(ref.sigma[:, None] - ref.sigma[None, :]) + np.diag(np.full(k, np.inf))
    gaps = gaps.min(axis=1) / ref.sigma
    bound = eps * ref.sigma[0] / (gaps * ref.sigma)
    gated = 0
    for i in range(k - 1):          # the gap below sigma_k is not known
        au = oracle.subspace_angles(U[:, i:i + 1], ref.U[:, i:i + 1])[0]
        av = oracle.subspace_angles(V[:, i:i + 1], ref.V[:, i:i + 1])[0]
        if bound[i] <= 1e-6:
            gated += 1
            assert au <= 1e-6 and av <= 1e-6, (i, au, av, bound[i])
        if bound[i] < 0.1:
            assert au <= 10 * bound[i] and av <= 10 * bound[i], (i, au, av, bound[i])
    assert gated >= 1 or bound[0] > 1e-6


@pytest.mark.parametrize("fmt", PRECISIONS)
def test_mixed_products_layouts_beyond_4GiB(gk, fmt):
    # 50,000 x 350,000: both internal layouts of the block products hold more than
    # 2^32 bytes, so byte offsets and the layout builders' work-item counts exceed
    # 32 bits.  Checked on sampled rows and columns against the oracle, including
    # rows and SNPs whose offsets lie beyond 2^32.
    n, p = 50000, 350000
    ld = (n + 3) // 4
    rng = np.random.default_rng(11)
    block = rng.integers(0, 256, size=(1000, ld), dtype=np.uint8)
    packed = np.tile(block, (p // 1000, 1))
    op = oracle.PackedOperator(packed, n, p)
    ctx = gk.Context(dev(packed), n, p, 1, precision=prec(gk, fmt), block_width=8,
                     krylov_dim=32)
    W = rng.standard_normal((p, 8)) / np.sqrt(p)
    X = rng.standard_normal((n, 8)) / np.sqrt(n)
    Y = ctx.matmat_mixed(dev(W)).cpu().numpy()
    Z = ctx.rmatmat_mixed(dev(X)).cpu().numpy()
    ctx.close()
    rows = np.concatenate([[0, n - 1, n - 2], rng.choice(n, 13, replace=False)])
    cols = np.concatenate([[0, p - 1, 345000, 349000], rng.choice(p, 12, replace=False)])
    for c in (0, 7):
        yr = op.matvec_rows(W[:, c], rows)
        zr = op.rmatvec_cols(X[:, c], cols)
        assert np.max(np.abs(Y[rows, c] - yr)) <= 1e-4 * np.max(np.abs(yr))
        assert np.max(np.abs(Z[cols, c] - zr)) <= 1e-4 * np.max(np.abs(zr))


@pytest.mark.parametrize("fmt", PRECISIONS)
def test_mixed_solve_recovers_planted_spikes(gk, fmt):
    # the spiked recipe (noise bulk + ten planted spikes at 1.5..20x the bulk edge)
    # at 4,000 x 40,000: the blocked solve matches the oracle to 1e-6 and every
    # planted spike stands clear of the bulk edge
    g = synth.config("c5", n=4000, p=40000)
    k = 10
    op, ref = _oracle(g, k)
    ctx = gk.Context(dev(g.packed), g.n, g.p, k, tol=1e-9, precision=prec(gk, fmt),
                     block_width=8)
    sigma, U, V, st, info = ctx.solve()
    ctx.close()
    assert st == gk.GKL_OK
    sigma = sigma.cpu().numpy()
    assert np.max(np.abs(sigma - ref.sigma) / ref.sigma) <= 1e-6
    assert np.all(sigma > 1.05 * g.meta["edge"])
