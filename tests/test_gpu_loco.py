"""Leave-one-block-out (LOCO) PCAs through the C ABI, against the oracle run on
each leave-one-out matrix.

Every problem of a LOCO batch is the whole matrix without one SNP block; the
library solves all of them together with block products on the matrix cores
(split BF16), so the tolerances are those of the mixed path:
  * sigma within 1e-6 relative of the oracle's for the same leave-one-out matrix
    (the oracle's standardisation is per column, so the leave-one-out matrix is
    the whole matrix's columns minus the block);
  * the right vectors are exactly zero on the problem's own block;
  * vectors under the gap rule of the mixed path: within 1e-6 rad where
    eps sigma_1 / (delta_i sigma_i) <= 1e-6, within 10 times that bound where it
    is below 0.1, eps = tol + the measured error of the block products.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def vec_angles(X, Y):
    c = np.sum(X * Y, axis=0)
    r = X - Y * c[None, :]
    return np.arctan2(np.linalg.norm(r, axis=0), np.abs(c))


def genome(n, sizes):
    blocks = [synth.config("c4", n=n, p=pc, chrom=c) for c, pc in sizes]
    packed = np.concatenate([b.packed for b in blocks], axis=0)
    starts = np.cumsum([0] + [b.p for b in blocks])
    return packed, starts


@pytest.mark.parametrize("fmt", ["bf16", "int8"])
def test_loco_matches_oracle_per_block(gk, fmt):
    n = 1500
    packed, bs = genome(n, [(3, 1800), (9, 1300), (15, 1000), (21, 700)])
    p = int(bs[-1])
    nb, k, tol = len(bs) - 1, 5, 1e-9
    prec = gk.GKL_PREC_MIXED if fmt == "bf16" else gk.GKL_PREC_MIXED_INT8
    Gd = dev(packed)
    ctx = gk.LocoContext(Gd, n, p, bs, k, tol=tol, precision=prec, krylov_dim=40)
    sig, Us, Vs, st, infos = ctx.solve()
    ctx.close()
    assert st == gk.GKL_OK
    # error of the block products (same kernels) on random unit vectors
    full = oracle.PackedOperator(packed, n, p)
    bctx = gk.Context(Gd, n, p, 1, precision=prec, block_width=8)
    rng = np.random.default_rng(5)
    W = rng.standard_normal((p, 4))
    W /= np.linalg.norm(W, axis=0)
    X = rng.standard_normal((n, 4))
    X /= np.linalg.norm(X, axis=0)
    dY = bctx.matmat_mixed(dev(W)).cpu().numpy() - np.stack([full.matvec(W[:, c]) for c in range(4)], 1)
    dZ = bctx.rmatmat_mixed(dev(X)).cpu().numpy() - np.stack([full.rmatvec(X[:, c]) for c in range(4)], 1)
    bctx.close()
    err = max(np.linalg.norm(dY, axis=0).max(), np.linalg.norm(dZ, axis=0).max())
    for q in range(nb):
        keep = np.concatenate([packed[bs[c]:bs[c + 1]] for c in range(nb) if c != q])
        op = oracle.PackedOperator(keep, n, keep.shape[0])
        ref = oracle.gkl_svd(op, k, tol=1e-12, v0=synth.start_vector(keep.shape[0], 5))
        s = sig[q].cpu().numpy()
        U = Us[q].cpu().numpy()
        V = Vs[q].cpu().numpy()
        assert infos[q].converged == 1
        assert np.max(np.abs(s - ref.sigma) / ref.sigma) <= 1e-6, (q, s, ref.sigma)
        assert np.all(V[bs[q]:bs[q + 1]] == 0.0)
        Vr = np.delete(V, np.arange(bs[q], bs[q + 1]), axis=0)
        eps = tol + err / ref.sigma[0]
        gaps = np.abs(ref.sigma[:, None] - ref.sigma[None, :]) + np.diag(np.full(k, np.inf))
        gaps = gaps.min(axis=1) / ref.sigma
        bound = eps * ref.sigma[0] / (gaps * ref.sigma)
        au, av = vec_angles(U, ref.U), vec_angles(Vr, ref.V)
        for i in range(k - 1):
            if bound[i] <= 1e-6:
                assert au[i] <= 1e-6 and av[i] <= 1e-6, (q, i, au[i], av[i], bound[i])
            if bound[i] < 0.1:
                assert au[i] <= 10 * bound[i] and av[i] <= 10 * bound[i], (q, i, au[i], av[i])


def test_loco_rejects_fp64_and_bad_blocks(gk):
    packed, bs = genome(400, [(20, 500), (21, 400)])
    Gd = dev(packed)
    p = int(bs[-1])
    with pytest.raises(gk.GKLError) as e:
        gk.LocoContext(Gd, 400, p, bs, 3, precision=gk.GKL_PREC_FP64)
    assert e.value.status == gk.GKL_ERR_UNSUPPORTED
    with pytest.raises(gk.GKLError) as e:
        gk.LocoContext(Gd, 400, p, [0, 500, 400, p], 3, precision=gk.GKL_PREC_MIXED)
    assert e.value.status == gk.GKL_ERR_INVALID
