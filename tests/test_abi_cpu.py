"""The C-ABI library loads and exports every declared entry point; argument
validation happens before any device call (runs without a GPU)."""
import ctypes

import pytest

import paper_1808_03374_amd as gk


def test_every_declared_symbol_is_exported():
    names = gk.declared_functions()
    assert "gkl_create" in names and "gkl_solve" in names and "gkl_destroy" in names
    assert len(names) >= 15
    for name in names:
        assert hasattr(gk.lib, name), f"libgkl.so does not export {name}"


def test_options_default_and_status_strings():
    o = gk.gkl_options_default()
    assert o.struct_size == ctypes.sizeof(gk.gkl_options)
    assert o.pro_omega == 1e-8 and o.krylov_dim == 0 and o.precision == gk.GKL_PREC_FP64
    for s in range(8):
        assert gk.gkl_status_string(s)
    assert gk.gkl_status_string(gk.GKL_NOT_CONVERGED) == "not converged"


FAKE = 0x1000   # never dereferenced: validation rejects before any device access


@pytest.mark.parametrize("args,msg", [
    ((FAKE, 0, 10, 1, 1e-8, 0), "n and p"),
    ((FAKE, 10, 0, 1, 1e-8, 0), "n and p"),
    ((FAKE, 10, 10, 0, 1e-8, 0), "k must"),
    ((FAKE, 10, 10, 11, 1e-8, 0), "k must"),
    ((FAKE, 10, 10, 2, 0.0, 0), "tol"),
    ((FAKE, 10, 10, 2, -1.0, 0), "tol"),
    ((FAKE, 10, 10, 2, 1e-8, 7), "reorth"),
    ((None, 10, 10, 2, 1e-8, 0), "G is NULL"),
])
def test_create_rejects_bad_arguments(args, msg):
    ctx = ctypes.c_void_p(12345)
    G, n, p, k, tol, re = args
    st = gk.lib.gkl_create(G, n, p, k, tol, re, ctypes.byref(ctx))
    assert st == gk.GKL_ERR_INVALID
    assert ctx.value == 12345            # no side effect on failure
    assert msg in gk.gkl_last_error(None)


@pytest.mark.parametrize("field,value,msg", [
    ("krylov_dim", 3, "krylov_dim"),
    ("krylov_dim", -1, "krylov_dim"),
    ("ld_bytes", 2, "ld_bytes"),
    ("block_width", 33, "block_width"),
    ("precision", 5, "precision"),
    ("precision", 4, "precision"),
    ("precision", -1, "precision"),
    ("keep", 1, "keep"),
])
def test_create_ex_rejects_bad_options(field, value, msg):
    o = gk.gkl_options_default()
    if field == "keep":
        o.krylov_dim = 20
    setattr(o, field, value)
    ctx = ctypes.c_void_p()
    st = gk.lib.gkl_create_ex(FAKE, 40, 50, 4, 1e-8, 0, ctypes.byref(o), ctypes.byref(ctx))
    assert st == gk.GKL_ERR_INVALID and msg in gk.gkl_last_error(None)


def test_struct_size_mismatch_is_rejected():
    o = gk.gkl_options_default()
    o.struct_size = 8
    ctx = ctypes.c_void_p()
    st = gk.lib.gkl_create_ex(FAKE, 40, 50, 4, 1e-8, 0, ctypes.byref(o), ctypes.byref(ctx))
    assert st == gk.GKL_ERR_INVALID


def test_null_safe_destroy_and_solve():
    gk.lib.gkl_destroy(None)
    info = gk.gkl_info()
    assert gk.lib.gkl_solve(None, None, None, 0, None, 0, ctypes.byref(info)) == gk.GKL_ERR_INVALID
    assert gk.lib.gkl_dense_svd(None, 4, None, None, None, None) == gk.GKL_ERR_INVALID
    assert gk.lib.gkl_dense_svd(FAKE, 0, FAKE, FAKE, FAKE, None) == gk.GKL_ERR_INVALID


def _batched(count, ns, ps, k=2, tol=1e-8, reorth=0, **fields):
    o = gk.gkl_options_default()
    for key, val in fields.items():
        setattr(o, key, val)
    G = (ctypes.c_void_p * max(count, 1))(*([FAKE] * max(count, 1)))
    N = (ctypes.c_int64 * max(count, 1))(*ns)
    P = (ctypes.c_int64 * max(count, 1))(*ps)
    ctx = ctypes.c_void_p(777)
    st = gk.lib.gkl_create_batched(count, G, N, P, k, tol, reorth, ctypes.byref(o), ctypes.byref(ctx))
    assert ctx.value == 777               # untouched on failure
    return st, gk.gkl_last_error(None)


@pytest.mark.parametrize("args,fields,status,msg", [
    ((0, [10], [10]), {}, gk.GKL_ERR_INVALID, "count"),
    ((1025, [10] * 1025, [10] * 1025), {}, gk.GKL_ERR_INVALID, "count"),
    ((2, [10, 0], [10, 10]), {}, gk.GKL_ERR_INVALID, "n and p"),
    ((2, [10, 10], [10, 3]), {}, gk.GKL_ERR_INVALID, "k must"),
    ((1, [10], [10]), {"krylov_dim": 2}, gk.GKL_ERR_INVALID, "krylov_dim"),
    ((1, [10], [10]), {"precision": 1}, gk.GKL_ERR_UNSUPPORTED, "FP64"),
    ((1, [10], [10]), {"precision": 2}, gk.GKL_ERR_UNSUPPORTED, "FP64"),
])
def test_create_batched_rejects_bad_arguments(args, fields, status, msg):
    count, ns, ps = args
    k = 4 if msg == "k must" else 2
    st, err = _batched(count, ns, ps, k=k, **fields)
    assert st == status and msg in err


def test_create_batched_partial_reorth_is_unsupported():
    st, err = _batched(1, [10], [10], reorth=1)
    assert st == gk.GKL_ERR_UNSUPPORTED and "full" in err


def test_batched_entry_points_reject_null():
    assert gk.lib.gkl_solve_batched(None, None, None, None, None, None, None) == gk.GKL_ERR_INVALID
    assert gk.lib.gkl_batched_plan(None, None, None, None, None, None, None) == gk.GKL_ERR_INVALID


@pytest.mark.parametrize("reorth,precision,restart,status,msg", [
    (0, 0, 7, gk.GKL_ERR_INVALID, "restart must"),
    (0, 0, -1, gk.GKL_ERR_INVALID, "restart must"),
    (1, 0, gk.GKL_RESTART_HARMONIC, gk.GKL_ERR_UNSUPPORTED, "harmonic"),
    (2, 0, gk.GKL_RESTART_HARMONIC, gk.GKL_ERR_UNSUPPORTED, "harmonic"),
    (0, 1, gk.GKL_RESTART_HARMONIC, gk.GKL_ERR_UNSUPPORTED, "harmonic"),
    (0, 3, gk.GKL_RESTART_HARMONIC, gk.GKL_ERR_UNSUPPORTED, "harmonic"),
])
def test_create_ex_checks_the_restart_option(reorth, precision, restart, status, msg):
    # the restart field sits where the binding puts it: the library reads back
    # the values written through ctypes
    o = gk.gkl_options_default()
    o.krylov_dim = 20
    o.precision = precision
    o.restart = restart
    ctx = ctypes.c_void_p()
    st = gk.lib.gkl_create_ex(FAKE, 40, 50, 4, 1e-8, reorth, ctypes.byref(o), ctypes.byref(ctx))
    assert st == status and msg in gk.gkl_last_error(None)


def test_create_batched_rejects_harmonic_restarts():
    st, err = _batched(1, [10], [10], restart=gk.GKL_RESTART_HARMONIC)
    assert st == gk.GKL_ERR_UNSUPPORTED and "harmonic" in err
