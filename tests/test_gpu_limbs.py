"""GPU parity of the FP64 products formed on the int8 matrix cores
(options.fp64_products = GKL_FP64_LIMBS) and of solves that use them.

Error model: the vector is scaled by a power of two 2^e at least its largest
magnitude (for A v: of (3 - mu_j) s_j v_j), rounded to an integer of at most 52
bits and split into seven 8-bit limbs whose sums are exact; each K split's
partial is recombined with one FP64 rounding and the splits are added in FP64.
Per output element the error is therefore at most 2^-53 2^e sum_j |c_ij| (the
quantisation, c = code) plus the roundings of an FP64 sum -- the same order as
the lookup-table products, so the same tolerances apply: 1e-12 ||y|| for the
products, 1e-10 sigma_i for singular values against the oracle.
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


def gen(name, n, p, seed=None, ld=None, pad_mode=0):
    g = synth.config(name, n=n, p=p, seed=seed, ld=ld, pad_mode=pad_mode)
    return g, dev(g.packed)


def limb_ctx(gk, Gd, n, p, k=1, **kw):
    return gk.Context(Gd, n, p, k, fp64_products=gk.GKL_FP64_LIMBS, **kw)


SHAPES = [("c1", 1000, 5000, None, 0), ("c2", 37, 513, 20, -1), ("c5", 1001, 333, None, -1),
          ("c1", 1, 7, None, -1), ("c2", 4099, 65, 1100, -1), ("c3", 16, 1, None, 0),
          ("c2", 3000, 70000, None, -1)]


@pytest.mark.parametrize("name,n,p,ld,pad", SHAPES)
def test_limb_products_match_oracle(gk, name, n, p, ld, pad):
    g, Gd = gen(name, n, p, ld=ld, pad_mode=pad)
    ctx = limb_ctx(gk, Gd, n, p)
    op = oracle.PackedOperator(g.packed, n, p)
    rng = np.random.default_rng(n * 7 + p)
    for scale in (1.0, 1e-100, 1e100):
        v = rng.standard_normal(p) * scale
        u = rng.standard_normal(n) * scale
        y = ctx.matvec(dev(v)).cpu().numpy()
        z = ctx.rmatvec(dev(u)).cpu().numpy()
        y0 = op.matvec(v)
        z0 = op.rmatvec(u)
        sy, sz = quantisation_slack(g, v, u)
        assert np.linalg.norm(y - y0) <= 1e-12 * np.linalg.norm(y0) + sy
        assert np.linalg.norm(z - z0) <= 1e-12 * np.linalg.norm(z0) + sz
    ctx.close()


def test_limb_products_wide_dynamic_range(gk):
    # entries spread over twelve orders of magnitude, a zero vector, and a
    # vector with a single nonzero entry
    g, Gd = gen("c2", 2000, 9000)
    n, p = g.n, g.p
    ctx = limb_ctx(gk, Gd, n, p)
    op = oracle.PackedOperator(g.packed, n, p)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(p) * 10.0 ** rng.uniform(-12, 0, p)
    u = rng.standard_normal(n) * 10.0 ** rng.uniform(-12, 0, n)
    for a, b in ((v, u), (np.zeros(p), np.zeros(n))):
        y = ctx.matvec(dev(a)).cpu().numpy()
        z = ctx.rmatvec(dev(b)).cpu().numpy()
        y0, z0 = op.matvec(a), op.rmatvec(b)
        assert np.linalg.norm(y - y0) <= 1e-12 * np.linalg.norm(y0) + 0.0
        assert np.linalg.norm(z - z0) <= 1e-12 * np.linalg.norm(z0) + 0.0
    e = np.zeros(p)
    e[p // 3] = 0.75
    y = ctx.matvec(dev(e)).cpu().numpy()
    assert np.linalg.norm(y - op.matvec(e)) <= 1e-14 * np.linalg.norm(op.matvec(e)) + \
        quantisation_slack(g, e, np.zeros(n))[0]
    ctx.close()


def test_limb_and_table_products_agree(gk):
    # both FP64 formats on one matrix, several K splits each
    g, Gd = gen("c2", 6000, 60000)
    n, p = g.n, g.p
    a = limb_ctx(gk, Gd, n, p)
    b = gk.Context(Gd, n, p, 1, fp64_products=gk.GKL_FP64_LUT)
    rng = np.random.default_rng(8)
    v = dev(rng.standard_normal(p))
    u = dev(rng.standard_normal(n))
    ya, yb = a.matvec(v).cpu().numpy(), b.matvec(v).cpu().numpy()
    za, zb = a.rmatvec(u).cpu().numpy(), b.rmatvec(u).cpu().numpy()
    assert np.linalg.norm(ya - yb) <= 1e-13 * np.linalg.norm(yb)
    assert np.linalg.norm(za - zb) <= 1e-13 * np.linalg.norm(zb)
    # repeated calls give the same bits
    assert np.array_equal(ya.view(np.uint64), a.matvec(v).cpu().numpy().view(np.uint64))
    a.close()
    b.close()


def test_limb_products_full_size_sampled(gk):
    # the full 10,000 x 100,000 workload on sampled rows and columns
    g, Gd = gen("c2", None, None)
    n, p = g.n, g.p
    ctx = limb_ctx(gk, Gd, n, p)
    op = oracle.PackedOperator(g.packed, n, p)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(p)
    u = rng.standard_normal(n)
    y = ctx.matvec(dev(v)).cpu().numpy()
    z = ctx.rmatvec(dev(u)).cpu().numpy()
    rows = np.concatenate([[0, n - 1], rng.choice(n, 62, replace=False)])
    cols = np.concatenate([[0, p - 1], rng.choice(p, 62, replace=False)])
    assert np.max(np.abs(y[rows] - op.matvec_rows(v, rows))) <= 1e-12 * np.linalg.norm(y) / np.sqrt(n) * 10
    assert np.max(np.abs(z[cols] - op.rmatvec_cols(u, cols))) <= 1e-12 * np.linalg.norm(z) / np.sqrt(p) * 10
    assert abs(y.sum()) <= 1e-10 * np.abs(y).sum()
    ctx.close()


def test_limb_products_beyond_4GiB(gk):
    # 50,000 x 350,000: both tiled layouts exceed 2^32 bytes; sampled rows and
    # SNPs whose offsets lie beyond 2^32
    n, p = 50000, 350000
    ld = (n + 3) // 4
    rng = np.random.default_rng(11)
    block = rng.integers(0, 256, size=(1000, ld), dtype=np.uint8)
    packed = np.tile(block, (p // 1000, 1))
    op = oracle.PackedOperator(packed, n, p)
    ctx = limb_ctx(gk, dev(packed), n, p)
    v = rng.standard_normal(p) / np.sqrt(p)
    u = rng.standard_normal(n) / np.sqrt(n)
    y = ctx.matvec(dev(v)).cpu().numpy()
    z = ctx.rmatvec(dev(u)).cpu().numpy()
    ctx.close()
    rows = np.concatenate([[0, n - 1, n - 2], rng.choice(n, 13, replace=False)])
    cols = np.concatenate([[0, p - 1, 345000, 349000], rng.choice(p, 12, replace=False)])
    yr = op.matvec_rows(v, rows)
    zr = op.rmatvec_cols(u, cols)
    assert np.max(np.abs(y[rows] - yr)) <= 1e-12 * np.linalg.norm(y) / np.sqrt(n) * 10
    assert np.max(np.abs(z[cols] - zr)) <= 1e-12 * np.linalg.norm(z) / np.sqrt(p) * 10


def _oracle_solve(g, k, seed, tol=1e-12):
    op = oracle.PackedOperator(g.packed, g.n, g.p)
    res = oracle.gkl_svd(op, k, tol=tol, v0=synth.start_vector(g.p, seed),
                         spare_left=synth.spare_directions(g.n, 8, seed),
                         spare_right=synth.spare_directions(g.p, 8, seed))
    return op, res


@pytest.mark.parametrize("fmt", ["limbs", "lut+limbs"])
@pytest.mark.parametrize("reorth,m", [("partial", 60), ("full", 60), ("full", 0)])
def test_limb_solve_matches_oracle(gk, reorth, m, fmt):
    g, Gd = gen("c2", 2000, 20000)
    k = 20 if m else 10
    op, ref = _oracle_solve(g, k, 3)
    re = gk.GKL_REORTH_FULL if reorth == "full" else gk.GKL_REORTH_PARTIAL
    choice = gk.GKL_FP64_LIMBS if fmt == "limbs" else gk.GKL_FP64_LUT_LIMBS
    ctx = gk.Context(Gd, g.n, g.p, k, tol=1e-11, reorth=re, v0=dev(synth.start_vector(g.p, 3)),
                     krylov_dim=m, fp64_products=choice)
    sigma, U, V, st, info = ctx.solve()
    assert st == gk.GKL_OK, gk.gkl_last_error(ctx.ctx)
    ctx.close()
    sigma = sigma.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    assert np.all(np.abs(sigma - ref.sigma) <= 1e-10 * ref.sigma)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-7
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-7
    r1, r2, _ = oracle.certificate(op, sigma, U, V)
    assert max(r1.max(), r2.max()) <= 1e-9 * sigma[0]
    assert np.dot(V[:, 0], ref.V[:, 0]) > 0


def test_fp64_products_option_is_validated(gk):
    g, Gd = gen("c1", 200, 900)
    with pytest.raises(gk.GKLError) as e:
        gk.Context(Gd, g.n, g.p, 3, fp64_products=7)
    assert e.value.status == gk.GKL_ERR_INVALID


@pytest.mark.parametrize("choice,n,p,expect", [
    ("AUTO", 2000, 9000, "LUT"), ("AUTO", 4000, 249999, "LUT"), ("AUTO", 4000, 250000, "LIMBS"),
    ("AUTO", 40000, 110000, "LIMBS"), ("LUT", 40000, 110000, "LUT"),
    ("LIMBS", 200, 900, "LIMBS"), ("LUT_LIMBS", 200, 900, "LUT_LIMBS")])
def test_fp64_products_reported(gk, choice, n, p, expect):
    # the format a solve ran in is reported; GKL_FP64_AUTO takes the limbs for
    # both products from n p >= 1e9 on (random bytes: the choice depends on the
    # shape only)
    gen_ = torch.Generator(device="cuda").manual_seed(n + p)
    Gd = torch.randint(0, 256, (p, (n + 3) // 4), dtype=torch.uint8, device="cuda", generator=gen_)
    ctx = gk.Context(Gd, n, p, 2, tol=1e-6, krylov_dim=8, max_matvecs=64,
                     fp64_products=getattr(gk, "GKL_FP64_" + choice))
    _, _, _, st, info = ctx.solve()
    ctx.close()
    assert st in (gk.GKL_OK, gk.GKL_NOT_CONVERGED)
    assert info.matvecs > 0
    assert info.fp64_products == getattr(gk, "GKL_FP64_" + expect)
