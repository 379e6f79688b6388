"""gkl_dense_svd_noalloc against gkl_dense_svd through the C ABI.

The no-allocation variant runs the same kernels on the same input with its
working memory in a fixed device array, so its output must equal
gkl_dense_svd's bit for bit.  Two calls in a row, the second smaller, show that
what the first call left in the shared array does not leak into the second.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_1808_03374_amd as m
    return m


def _matrix(m, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((m, m))
    if m > 4:
        B = np.triu(np.tril(B, 1))
        B[0, m // 2] = 0.7
    return torch.from_numpy(B.T.copy()).cuda()


def _svd(fn, Bd, m):
    P = torch.empty((m, m), dtype=torch.float64, device="cuda")
    S = torch.empty(m, dtype=torch.float64, device="cuda")
    Q = torch.empty((m, m), dtype=torch.float64, device="cuda")
    fn(Bd, m, P, S, Q)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (P, S, Q)]


@pytest.mark.parametrize("sizes", [(200, 120), (128, 100), (256, 60)])
def test_noalloc_matches_allocating_call(gk, sizes):
    for i, m in enumerate(sizes):
        Bd = _matrix(m, 1000 + 7 * m + i)
        got = _svd(gk.gkl_dense_svd_noalloc, Bd, m)
        ref = _svd(gk.gkl_dense_svd, Bd, m)
        for a, b in zip(got, ref):
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), m
        # and it is an SVD of B
        P, S, Q = (got[0].T, got[1], got[2].T)
        B = Bd.cpu().numpy().T
        assert np.abs(P * S @ Q.T - B).max() < 1e-12 * S[0]


def test_noalloc_rejects_sizes_beyond_its_scratch(gk):
    m = 257
    Bd = _matrix(m, 3)
    with pytest.raises(gk.GKLError) as e:
        _svd(gk.gkl_dense_svd_noalloc, Bd, m)
    assert e.value.status == gk.GKL_ERR_INVALID
    assert "256" in str(e.value)
