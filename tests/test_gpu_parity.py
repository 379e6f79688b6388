"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances
  * decode, counts, mean, scale: bit-exact (integer work; mean and scale are
    single correctly rounded IEEE operations in a fixed order on both sides).
  * FP64 products: ||y_gpu - y_oracle|| <= 1e-12 ||y_oracle||.  Both sides sum
    p (or n) FP64 terms in different orders; the rounding difference is bounded by
    about sqrt(p) * eps * sum|terms| ~ 1e-14 ||y|| at these sizes, so 1e-12
    leaves two orders of magnitude of margin.
  * singular values: |sigma_gpu - sigma_oracle| <= 1e-10 sigma_i (FP64 path).
  * vectors: principal angle <= 1e-6 for singular values with a clear gap.
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


SHAPES = [("c1", 1000, 5000, None, 0), ("c2", 37, 513, 20, -1), ("c5", 1001, 333, None, -1),
          ("c1", 1, 7, None, -1), ("c2", 4099, 65, 1100, -1), ("c3", 16, 1, None, 0)]


@pytest.mark.parametrize("name,n,p,ld,pad", SHAPES)
def test_column_stats_bit_exact(gk, name, n, p, ld, pad):
    g, Gd = gen(name, n, p, ld=ld, pad_mode=pad)
    ctx = gk.Context(Gd, n, p, 1)
    count, nobs, mean, inv_sd = [t.cpu().numpy() for t in ctx.column_stats()]
    st = oracle.column_stats(n, *oracle.counts(g.packed, n, p))
    assert np.array_equal(count, st.count)
    assert np.array_equal(nobs, st.nobs)
    assert np.array_equal(mean.view(np.uint64), st.mean.view(np.uint64))
    assert np.array_equal(inv_sd.view(np.uint64), st.inv_sd.view(np.uint64))
    ctx.close()


def test_column_stats_special_columns(gk):
    n = 23
    codes = np.zeros((n, 6), dtype=np.int64)
    codes[:, 1] = 2                       # monomorphic
    codes[:, 2] = 3                       # all missing
    codes[:, 3] = np.arange(n) % 3        # 0,1,2
    codes[::4, 4] = 3
    codes[:, 5] = 1
    packed = synth.pack_codes(codes, ld=9, pad_mode=-1)
    ctx = gk.Context(dev(packed), n, 6, 1)
    count, nobs, mean, inv_sd = [t.cpu().numpy() for t in ctx.column_stats()]
    st = oracle.column_stats(n, *oracle.counts(packed, n, 6))
    assert np.array_equal(inv_sd.view(np.uint64), st.inv_sd.view(np.uint64))
    assert inv_sd[0] == 0 and inv_sd[1] == 0 and inv_sd[2] == 0 and mean[2] == 0
    ctx.close()


@pytest.mark.parametrize("name,n,p,ld,pad", SHAPES[:5])
def test_unpack_bit_exact(gk, name, n, p, ld, pad):
    g, Gd = gen(name, n, p, ld=ld, pad_mode=pad)
    ctx = gk.Context(Gd, n, p, 1)
    got = ctx.unpack().cpu().numpy()
    assert np.array_equal(got, oracle.decode(g.packed, n, p))
    ctx.close()


def test_hooks_on_a_blocked_context(gk):
    # unpack decodes the caller's matrix whatever the context kind; the FP64
    # product hooks need an FP64 context and say so
    g, Gd = gen("c2", 300, 2000, pad_mode=-1)
    ctx = gk.Context(Gd, g.n, g.p, 4, precision=gk.GKL_PREC_MIXED, block_width=8)
    got = ctx.unpack().cpu().numpy()
    assert np.array_equal(got, oracle.decode(g.packed, g.n, g.p))
    st = oracle.column_stats(g.n, *oracle.counts(g.packed, g.n, g.p))
    mean = ctx.column_stats()[2].cpu().numpy()
    assert np.array_equal(mean.view(np.uint64), st.mean.view(np.uint64))
    with pytest.raises(gk.GKLError) as e:
        ctx.matvec(dev(np.ones(g.p)))
    assert e.value.status == gk.GKL_ERR_INVALID and "FP64" in str(e.value)
    ctx.close()
    f64 = gk.Context(Gd, g.n, g.p, 4)
    with pytest.raises(gk.GKLError) as e:
        f64.matmat_mixed(dev(np.ones((g.p, 2))))
    assert e.value.status == gk.GKL_ERR_INVALID
    f64.close()


@pytest.mark.parametrize("fmt", ["lut", "lut+limbs"])
@pytest.mark.parametrize("name,n,p,ld,pad", SHAPES)
def test_matvec_parity(gk, name, n, p, ld, pad, fmt):
    # the lookup-table products, and the large-matrix default (tables for A v,
    # int8 limbs for A^T u, whose vector quantisation adds the bound of
    # limb_bounds)
    g, Gd = gen(name, n, p, ld=ld, pad_mode=pad)
    choice = gk.GKL_FP64_LUT if fmt == "lut" else gk.GKL_FP64_LUT_LIMBS
    ctx = gk.Context(Gd, n, p, 1, fp64_products=choice)
    op = oracle.PackedOperator(g.packed, n, p)
    rng = np.random.default_rng(n * 7 + p)
    v = rng.standard_normal(p)
    u = rng.standard_normal(n)
    y = ctx.matvec(dev(v)).cpu().numpy()
    z = ctx.rmatvec(dev(u)).cpu().numpy()
    y0 = op.matvec(v)
    z0 = op.rmatvec(u)
    sz = quantisation_slack(g, v, u)[1] if fmt != "lut" else 0.0
    assert np.linalg.norm(y - y0) <= 1e-12 * max(np.linalg.norm(y0), 1e-300)
    assert np.linalg.norm(z - z0) <= 1e-12 * max(np.linalg.norm(z0), 1e-300) + sz
    ctx.close()


def test_matvec_full_size_sampled(gk):
    # the full 10,000 x 100,000 workload, checked on sampled rows and columns
    g, Gd = gen("c2", None, None)
    n, p = g.n, g.p
    ctx = gk.Context(Gd, n, p, 1)
    op = oracle.PackedOperator(g.packed, n, p)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(p)
    u = rng.standard_normal(n)
    y = ctx.matvec(dev(v)).cpu().numpy()
    z = ctx.rmatvec(dev(u)).cpu().numpy()
    rows = np.concatenate([[0, n - 1], rng.choice(n, 62, replace=False)])
    cols = np.concatenate([[0, p - 1], rng.choice(p, 62, replace=False)])
    yr = op.matvec_rows(v, rows)
    zc = op.rmatvec_cols(u, cols)
    assert np.max(np.abs(y[rows] - yr)) <= 1e-12 * np.linalg.norm(y) / np.sqrt(n) * 10
    assert np.max(np.abs(z[cols] - zc)) <= 1e-12 * np.linalg.norm(z) / np.sqrt(p) * 10
    # centred columns: the scores sum to zero
    assert abs(y.sum()) <= 1e-10 * np.abs(y).sum()
    ctx.close()


@pytest.mark.parametrize("m", [1, 2, 7, 60, 96, 97, 112, 128, 129, 150])
def test_dense_svd(gk, m):
    rng = np.random.default_rng(m)
    B = rng.standard_normal((m, m))
    if m > 4:
        B = np.triu(np.tril(B, 1))      # bidiagonal-like, as in GKL
        B[0, m // 2] = 0.7              # plus a spike entry, as after a restart
    Bd = dev(B.T.copy())                 # column-major
    P = torch.empty((m, m), dtype=torch.float64, device="cuda")
    S = torch.empty(m, dtype=torch.float64, device="cuda")
    Q = torch.empty((m, m), dtype=torch.float64, device="cuda")
    gk.gkl_dense_svd(Bd, m, P, S, Q)
    P = P.cpu().numpy().T
    Q = Q.cpu().numpy().T
    S = S.cpu().numpy()
    s_ref = np.linalg.svd(B, compute_uv=False)
    assert np.all(np.abs(S - s_ref) <= 1e-13 * s_ref[0] * max(1, m / 10))
    assert np.abs(P.T @ P - np.eye(m)).max() < 1e-12
    assert np.abs(Q.T @ Q - np.eye(m)).max() < 1e-12
    assert np.abs(P * S @ Q.T - B).max() < 1e-12 * s_ref[0]


def _oracle_solve(g, k, seed, tol=1e-12):
    op = oracle.PackedOperator(g.packed, g.n, g.p)
    res = oracle.gkl_svd(op, k, tol=tol, v0=synth.start_vector(g.p, seed),
                         spare_left=synth.spare_directions(g.n, 8, seed),
                         spare_right=synth.spare_directions(g.p, 8, seed))
    return op, res


def _residuals(op, sigma, U, V):
    r1, r2, _ = oracle.certificate(op, sigma, U, V)
    return max(r1.max(), r2.max())


def test_gkl_full_reorth_small_config(gk):
    # 1,000 x 5,000, two subpopulations, k = 10, plain GKL with full CGS2
    g, Gd = gen("c1", None, None)
    k = 10
    op, ref = _oracle_solve(g, k, 1)
    v0 = dev(synth.start_vector(g.p, 1))
    ctx = gk.Context(Gd, g.n, g.p, k, tol=1e-12, reorth=gk.GKL_REORTH_FULL, v0=v0, trace=1,
                     check_every=1)
    sigma, U, V, st, info = ctx.solve()
    assert st == gk.GKL_OK and info.converged == 1
    sigma = sigma.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    assert np.all(np.abs(sigma - ref.sigma) <= 1e-10 * ref.sigma)
    # the recurrence scalars follow the oracle step by step
    tr = ctx.trace()
    steps = min(10, len(tr))
    assert np.allclose(tr[:steps, 1], ref.alphas[:steps], rtol=1e-12, atol=0)
    assert np.allclose(tr[:steps, 2], ref.betas[:steps], rtol=1e-12, atol=0)
    # vectors: orthonormal, residuals small, the leading (gapped) vector matches
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-12
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-12
    assert _residuals(op, sigma, U, V) <= 1e-9 * sigma[0]
    assert oracle.subspace_angles(V[:, :1], ref.V[:, :1]).max() < 1e-6
    assert oracle.subspace_angles(U[:, :1], ref.U[:, :1]).max() < 1e-6
    # same sign rule on both sides
    assert np.dot(V[:, 0], ref.V[:, 0]) > 0 and np.dot(U[:, 0], ref.U[:, 0]) > 0
    ctx.close()


@pytest.mark.parametrize("reorth", ["full", "partial"])
def test_gkl_thick_restart(gk, reorth):
    # the 5-subpopulation recipe at 2,000 x 20,000; k = 20 with a 60-vector basis
    g, Gd = gen("c2", 2000, 20000)
    k = 20
    op, ref = _oracle_solve(g, k, 3)
    v0 = dev(synth.start_vector(g.p, 3))
    re = gk.GKL_REORTH_FULL if reorth == "full" else gk.GKL_REORTH_PARTIAL
    ctx = gk.Context(Gd, g.n, g.p, k, tol=1e-11, reorth=re, v0=v0, krylov_dim=60)
    sigma, U, V, st, info = ctx.solve()
    assert st == gk.GKL_OK, gk.gkl_last_error(ctx.ctx)
    assert info.restarts >= 1
    sigma = sigma.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    assert np.all(np.abs(sigma - ref.sigma) <= 1e-10 * ref.sigma)
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-7
    assert _residuals(op, sigma, U, V) <= 1e-9 * sigma[0]
    gap = np.abs(np.diff(ref.sigma)) / ref.sigma[:-1]
    for i in range(k - 1):
        if gap[i] > 1e-2 and (i == 0 or gap[i - 1] > 1e-2):
            assert oracle.subspace_angles(V[:, i:i + 1], ref.V[:, i:i + 1]).max() < 1e-6
    ctx.close()


@pytest.mark.parametrize("reorth", ["full", "partial"])
def test_gkl_wide_basis_ragged(gk, reorth):
    # a 100-vector basis (more than 64 columns per Gram-Schmidt pass) on lengths
    # that are not multiples of the 64-row tiles: 1,300 x 7,000, k = 20
    g, Gd = gen("c2", 1300, 7000)
    k = 20
    op, ref = _oracle_solve(g, k, 5)
    v0 = dev(synth.start_vector(g.p, 5))
    re = gk.GKL_REORTH_FULL if reorth == "full" else gk.GKL_REORTH_PARTIAL
    ctx = gk.Context(Gd, g.n, g.p, k, tol=1e-11, reorth=re, v0=v0, krylov_dim=100)
    sigma, U, V, st, info = ctx.solve()
    assert st == gk.GKL_OK, gk.gkl_last_error(ctx.ctx)
    sigma = sigma.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    assert np.all(np.abs(sigma - ref.sigma) <= 1e-10 * ref.sigma)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-7
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-7
    assert _residuals(op, sigma, U, V) <= 1e-9 * sigma[0]
    ctx.close()


def test_two_group_closed_form_and_rank_deficiency(gk):
    n, p = 40, 30
    codes = np.zeros((n, p), dtype=np.int64)
    codes[n // 2:] = 2
    packed = synth.pack_codes(codes)
    ctx = gk.Context(dev(packed), n, p, 3, tol=1e-12, v0=dev(synth.start_vector(p, 0)))
    sigma, U, V, st, info = ctx.solve()
    sigma = sigma.cpu().numpy()
    assert abs(sigma[0] - np.sqrt(2.0 * n * p)) <= 1e-12 * np.sqrt(2.0 * n * p)
    assert np.all(np.abs(sigma[1:]) <= 1e-9 * sigma[0])
    ctx.close()


def test_not_converged_still_writes_output(gk):
    g, Gd = gen("c1", 300, 900)
    ctx = gk.Context(Gd, g.n, g.p, 5, tol=1e-14, max_matvecs=6)
    sigma, U, V, st, info = ctx.solve()
    assert st == gk.GKL_NOT_CONVERGED and info.converged == 0
    assert np.all(np.isfinite(sigma.cpu().numpy())) and info.matvecs <= 8
    ctx.close()


def test_solve_is_deterministic(gk):
    g, Gd = gen("c2", 700, 3000)
    ctx = gk.Context(Gd, g.n, g.p, 6, tol=1e-10, krylov_dim=24, reorth=gk.GKL_REORTH_PARTIAL)
    a = [t.cpu().numpy().copy() for t in ctx.solve()[:3]]
    b = [t.cpu().numpy().copy() for t in ctx.solve()[:3]]
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint64), y.view(np.uint64))
    ctx.close()


@pytest.mark.parametrize("stride", [1, 3])
def test_product_timing_sampling(gk, stride):
    # options.timing = t brackets the first of every t launches of each product;
    # the results do not depend on it
    g, Gd = gen("c2", 700, 3000)
    base = gk.Context(Gd, g.n, g.p, 6, tol=1e-10, krylov_dim=24, reorth=gk.GKL_REORTH_PARTIAL)
    s0, _, _, _, i0 = base.solve()
    base.close()
    ctx = gk.Context(Gd, g.n, g.p, 6, tol=1e-10, krylov_dim=24, reorth=gk.GKL_REORTH_PARTIAL,
                     timing=stride)
    s1, _, _, _, i1 = ctx.solve()
    ctx.close()
    assert torch.equal(s0, s1)
    n_mv = i1.matvecs // 2 + i1.matvecs % 2    # A v comes first in every step
    n_rmv = i1.matvecs // 2
    assert i1.timed_matvecs == -(-n_mv // stride)
    assert i1.timed_rmatvecs == -(-n_rmv // stride)
    assert i0.timed_matvecs == 0 and i0.matvec_kernel_ms == 0.0
    assert i1.matvec_kernel_ms > 0.0 and i1.rmatvec_kernel_ms > 0.0


@pytest.mark.parametrize("name,n,p,k,m", [("c1", 1000, 5000, 10, 0), ("c2", 2000, 20000, 20, 60),
                                          ("c3", 3000, 1500, 10, 40)])
def test_one_sided_reorthogonalisation(gk, name, n, p, k, m):
    # Section 3, "Choice of reorthogonalization strategy": Gram-Schmidt on the
    # shorter side only (U for n <= p, V for the tall 3,000 x 1,500 case), the
    # longer side's vectors recomputed from it at the end; sigma must match the
    # oracle as with full reorthogonalisation
    g, Gd = gen(name, n, p)
    op, ref = _oracle_solve(g, k, 2)
    v0 = dev(synth.start_vector(g.p, 2))
    runs = {}
    for mode in (gk.GKL_REORTH_FULL, gk.GKL_REORTH_ONESIDED):
        ctx = gk.Context(Gd, g.n, g.p, k, tol=1e-11, reorth=mode, v0=v0, krylov_dim=m)
        runs[mode] = ctx.solve()
        ctx.close()
    sigma, U, V, st, info = runs[gk.GKL_REORTH_ONESIDED]
    assert st == gk.GKL_OK
    full = runs[gk.GKL_REORTH_FULL][4]
    assert info.reorths < full.reorths, (info.reorths, full.reorths)
    sigma = sigma.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    assert np.all(np.abs(sigma - ref.sigma) <= 1e-10 * ref.sigma)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-9
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-9
    assert _residuals(op, sigma, U, V) <= 1e-9 * sigma[0]
    # same sign rule as the oracle on the leading (gapped) vector
    assert np.dot(V[:, 0], ref.V[:, 0]) > 0


def test_one_sided_is_fp64_only(gk):
    g, Gd = gen("c1", 200, 900)
    with pytest.raises(gk.GKLError) as e:
        gk.Context(Gd, g.n, g.p, 3, reorth=gk.GKL_REORTH_ONESIDED, precision=gk.GKL_PREC_MIXED,
                   block_width=4)
    assert e.value.status == gk.GKL_ERR_UNSUPPORTED


def test_gkl_without_restart_past_the_lds_basis(gk):
    # no restart, 2,000 x 20,000, k = 20 to 1e-12: the basis grows past 128
    # columns, so the convergence tests run the Ritz SVD whose sweeps are spread
    # over workgroups (the projected matrix no longer fits LDS)
    g, Gd = gen("c2", 2000, 20000)
    k = 20
    op = oracle.PackedOperator(g.packed, g.n, g.p)
    ref = oracle.gkl_svd(op, k, tol=1e-12, v0=synth.start_vector(g.p, 7),
                         spare_left=synth.spare_directions(g.n, 8, 7),
                         spare_right=synth.spare_directions(g.p, 8, 7), check_every=50)
    ctx = gk.Context(Gd, g.n, g.p, k, tol=1e-12, reorth=gk.GKL_REORTH_FULL,
                     v0=dev(synth.start_vector(g.p, 7)))
    sigma, U, V, st, info = ctx.solve()
    ctx.close()
    assert st == gk.GKL_OK and info.steps > 128, (st, info.steps)
    sigma = sigma.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    assert np.all(np.abs(sigma - ref.sigma) <= 1e-10 * ref.sigma)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-10
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-10
    assert _residuals(op, sigma, U, V) <= 1e-9 * sigma[0]
