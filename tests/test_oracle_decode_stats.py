"""Oracle pins: decode, counts, column statistics, the standardised matrix."""
import os

import numpy as np
import pytest

import oracle
import synth
from conftest import GOLDEN


def _golden_bytes():
    rows = []
    with open(os.path.join(GOLDEN, "decode_bytes.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                parts = line.split()
                rows.append((int(parts[0], 16), [int(x) for x in parts[1:]]))
    return rows


def test_decode_golden_bytes():
    rows = _golden_bytes()
    assert len(rows) >= 10
    packed = np.array([[b] for b, _ in rows], dtype=np.uint8)      # p columns of n = 4
    got = oracle.decode(packed, 4, len(rows))
    for j, (_, want) in enumerate(rows):
        assert got[:, j].tolist() == want


def test_decode_all_bytes_roundtrip():
    packed = np.arange(256, dtype=np.uint8).reshape(256, 1)
    got = oracle.decode(packed, 4, 256).astype(np.int64)
    code = np.where(got < 0, 3, got)
    rebuilt = sum(code[k, :] * 4 ** k for k in range(4))
    assert np.array_equal(rebuilt, np.arange(256))


@pytest.mark.parametrize("n", [1, 5, 37, 64, 129])
def test_decode_ignores_padding(n):
    rng = np.random.default_rng(n)
    codes = rng.integers(0, 4, size=(n, 11))
    clean = synth.pack_codes(codes, pad_mode=0)
    dirty = synth.pack_codes(codes, ld=(n + 3) // 4 + 7, pad_mode=-1)
    want = np.where(codes == 3, -1, codes)
    assert np.array_equal(oracle.decode(clean, n, 11), want)
    assert np.array_equal(oracle.decode(dirty, n, 11), want)
    c1 = oracle.counts(dirty, n, 11)
    for c, arr in zip((1, 2, 3), c1):
        assert np.array_equal(arr, np.sum(codes == c, axis=0))


def test_counts_match_decode_on_generated_data():
    g = synth.config("c1", n=203, p=517)
    codes = oracle.decode(g.packed, g.n, g.p)
    n1, n2, n3 = oracle.counts(g.packed, g.n, g.p)
    assert np.array_equal(n1, np.sum(codes == 1, axis=0))
    assert np.array_equal(n2, np.sum(codes == 2, axis=0))
    assert np.array_equal(n3, np.sum(codes == -1, axis=0))


def _stats_of(cols):
    codes = np.array(cols, dtype=np.int64).T          # n x p, 3 = missing
    n = codes.shape[0]
    n1 = np.sum(codes == 1, axis=0)
    n2 = np.sum(codes == 2, axis=0)
    n3 = np.sum(codes == 3, axis=0)
    return oracle.column_stats(n, n1, n2, n3)


def test_column_stats_closed_forms():
    st = _stats_of([[1, 1, 1, 1],        # f = 1/2: mu = 1, s = sqrt(2)
                    [0, 0, 0, 0],        # monomorphic: s = 0
                    [2, 2, 2, 2],        # monomorphic: s = 0
                    [3, 3, 3, 3],        # all missing: mu = 0, s = 0
                    [0, 2, 0, 2],        # mu = 1, s = sqrt(2)
                    [1, 1, 3, 2],        # mu = 4/3, var = 4/9, s = 3/2
                    [0, 0, 0, 1]])       # mu = 1/4, var = 7/32
    assert st.count.tolist() == [4, 0, 8, 0, 4, 4, 1]
    assert st.nobs.tolist() == [4, 4, 4, 0, 4, 3, 4]
    ulp = np.spacing(np.sqrt(2.0))
    assert st.mean[0] == 1.0 and abs(st.inv_sd[0] - np.sqrt(2.0)) <= ulp
    assert st.inv_sd[1] == 0.0 and st.inv_sd[2] == 0.0
    assert st.mean[3] == 0.0 and st.inv_sd[3] == 0.0
    assert st.inv_sd[4] == st.inv_sd[0]
    assert st.mean[5] == 4.0 / 3.0
    assert abs(st.inv_sd[5] - 1.5) <= 2e-16 * 1.5
    assert abs(st.inv_sd[6] - np.sqrt(32.0 / 7.0)) <= 4e-16 * np.sqrt(32.0 / 7.0)


def test_standardised_column_by_hand():
    # one SNP over individuals with codes 0, 1, 2, missing: mu = 1, s = sqrt 2
    packed = synth.pack_codes(np.array([[0], [1], [2], [3]]))
    op = oracle.PackedOperator(packed, 4, 1)
    col = op.matvec(np.array([1.0]))
    r2 = np.sqrt(2.0)
    assert np.allclose(col, [-r2, 0.0, r2, 0.0], rtol=0, atol=1e-15)
    z = op.rmatvec(np.array([1.0, 10.0, 100.0, 1000.0]))
    assert np.allclose(z, [-r2 + 100 * r2], rtol=1e-15)


def test_frobenius_from_counts():
    g = synth.config("c1", n=150, p=400)
    codes = oracle.decode(g.packed, g.n, g.p)
    st = oracle.column_stats(g.n, *oracle.counts(g.packed, g.n, g.p))
    A = oracle.dense_matrix(codes, st.mean, st.inv_sd)
    assert abs(np.sum(A * A) - oracle.frobenius_sq_from_counts(st)) <= 1e-11 * np.sum(A * A)
