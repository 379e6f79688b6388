"""Planted mistakes in the oracle (on the CPU): each must be caught by a pin.

A pin that passes with a plausible mistake planted in the oracle is not a pin.
Each case patches one oracle function with a wrong variant and re-runs the
pin that should catch it.
"""
import numpy as np
import pytest

import oracle
import oracle.gkl_oracle as og
import synth


def _two_group_sigma():
    n, p = 40, 30
    codes = np.zeros((n, p), dtype=np.int64)
    codes[n // 2:] = 2
    packed = synth.pack_codes(codes)
    st = og.column_stats(n, *og.counts(packed, n, p))
    A = og.dense_matrix(og.decode(packed, n, p), st.mean, st.inv_sd)
    res = og.gkl_svd(og.DenseOperator(A), 1, tol=1e-13, v0=synth.start_vector(p, 0),
                     spare_left=synth.spare_directions(n, 4, 0),
                     spare_right=synth.spare_directions(p, 4, 0))
    return res.sigma[0], np.sqrt(2.0 * n * p)


def _dense_pin():
    g = synth.config("c1", n=200, p=500)
    st = og.column_stats(g.n, *og.counts(g.packed, g.n, g.p))
    A = og.dense_matrix(og.decode(g.packed, g.n, g.p), st.mean, st.inv_sd)
    try:
        res = og.gkl_svd(og.DenseOperator(A), 6, tol=1e-12, v0=synth.start_vector(g.p, 1),
                         max_steps=200)
    except RuntimeError:          # a mutant that breaks down fails the pin too
        return False
    s = np.linalg.svd(A, compute_uv=False)[:6]
    ok_sigma = np.all(np.abs(res.sigma - s) <= 1e-10 * s[0])
    R = A @ res.V - res.U * res.sigma
    ok_vec = np.linalg.norm(R, axis=0).max() <= 1e-9 * s[0]
    return bool(ok_sigma and ok_vec)


def _hand_column_pin():
    codes = np.array([[0], [1], [2], [-1]])
    st = og.column_stats(4, np.array([1]), np.array([1]), np.array([1]))
    col = og.dense_matrix(codes, st.mean, st.inv_sd)[:, 0]
    r2 = np.sqrt(2.0)
    return bool(np.allclose(col, [-r2, 0.0, r2, 0.0], atol=1e-15))


def test_pins_pass_unmutated():
    s, want = _two_group_sigma()
    assert abs(s - want) <= 1e-12 * want
    assert _dense_pin()
    assert _hand_column_pin()


def test_sample_sd_scaling_is_caught(monkeypatch):
    orig = og.column_stats

    def wrong(n, n1, n2, n3):
        st = orig(n, n1, n2, n3)
        sumsq = (np.asarray(n1) + 4 * np.asarray(n2)).astype(float)
        var = sumsq / st.nobs - st.mean ** 2          # sample variance instead of 2f(1-f)
        st.inv_sd = np.where(var > 0, 1.0 / np.sqrt(np.where(var > 0, var, 1.0)), 0.0)
        return st

    monkeypatch.setattr(og, "column_stats", wrong)
    s, want = _two_group_sigma()
    assert abs(s - want) > 1e-3 * want


def test_unmasked_missing_is_caught(monkeypatch):
    def wrong(codes, mean, inv_sd):
        g = np.where(codes < 0, 3, codes).astype(np.float64)   # missing read as code 3
        return (g - mean[None, :]) * inv_sd[None, :]

    monkeypatch.setattr(og, "dense_matrix", wrong)
    assert not _hand_column_pin()


def test_transposed_bidiagonal_is_caught(monkeypatch):
    orig = og._bidiag
    monkeypatch.setattr(og, "_bidiag", lambda a, b: orig(a, b).T)
    assert not _dense_pin()


def test_wrong_sign_gram_schmidt_is_caught(monkeypatch):
    def wrong(Q, r):
        if Q.shape[1] == 0:
            return r
        r = r + Q @ (Q.T @ r)          # projection added instead of removed
        return r + Q @ (Q.T @ r)

    monkeypatch.setattr(og, "cgs2", wrong)
    assert not _dense_pin()
