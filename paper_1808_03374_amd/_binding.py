"""ctypes marshalling for libgkl.so; names mirror include/gkl.h."""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libgkl.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "gkl.h")

GKL_OK = 0
GKL_ERR_INVALID = 1
GKL_ERR_NOMEM = 2
GKL_ERR_DEVICE = 3
GKL_NOT_CONVERGED = 4
GKL_ERR_BREAKDOWN = 5
GKL_ERR_INTERNAL = 6
GKL_ERR_UNSUPPORTED = 7
GKL_REORTH_FULL = 0
GKL_REORTH_PARTIAL = 1
GKL_REORTH_ONESIDED = 2
GKL_PREC_FP64 = 0
GKL_PREC_MIXED = 1
GKL_PREC_MIXED_INT8 = 2
GKL_PREC_BLOCK_FP64 = 3
GKL_FP64_AUTO = 0
GKL_FP64_LUT = 1
GKL_FP64_LIMBS = 2
GKL_FP64_LUT_LIMBS = 3
GKL_TRACE_FIELDS = 7
GKL_RESTART_RITZ = 0
GKL_RESTART_HARMONIC = 1


class gkl_options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("krylov_dim", ctypes.c_int32),
        ("keep", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("block_width", ctypes.c_int32),
        ("adaptive_cgs2", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("max_steps", ctypes.c_int32),
        ("pro_omega", ctypes.c_double),
        ("max_matvecs", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("v0", ctypes.c_void_p),
        ("ld_bytes", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("trace", ctypes.c_int32),
        ("verbose", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("fp64_products", ctypes.c_int32),
        ("restart", ctypes.c_int32),
    ]


class gkl_info(ctypes.Structure):
    _fields_ = [
        ("matvecs", ctypes.c_int64),
        ("passes_over_G", ctypes.c_int64),
        ("steps", ctypes.c_int64),
        ("restarts", ctypes.c_int64),
        ("reorths", ctypes.c_int64),
        ("nconv", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("sum_residual_est", ctypes.c_double),
        ("max_residual_rel", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
        ("create_ms", ctypes.c_double),
        ("matvec_kernel_ms", ctypes.c_double),
        ("rmatvec_kernel_ms", ctypes.c_double),
        ("timed_matvecs", ctypes.c_int64),
        ("timed_rmatvecs", ctypes.c_int64),
        ("matvec_core_ms", ctypes.c_double),
        ("rmatvec_core_ms", ctypes.c_double),
        ("fp64_products", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class GKLError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{gkl_status_string(status)} ({status}): {message}")
        self.status = status


if not os.path.exists(library_path):
    raise ImportError(
        f"{library_path} is missing: build it with paper_1808_03374_amd/build.py "
        "(or __graft_entry__.build()); there is no non-HIP fallback")

# torch ships its own HIP runtime whose file name differs from the soname that
# libgkl.so records.  Loading libgkl.so first would pull in a second HIP/HSA
# runtime, and whichever initialises second finds no device.  Importing torch
# first makes libgkl.so bind to the runtime torch already holds.
try:
    import torch  # noqa: F401
except ImportError:
    torch = None

lib = ctypes.CDLL(library_path)

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_st = ctypes.c_int
_ctx_pp = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "gkl_options_default": (None, [ctypes.POINTER(gkl_options)]),
    "gkl_status_string": (ctypes.c_char_p, [_st]),
    "gkl_last_error": (ctypes.c_char_p, [_vp]),
    "gkl_create": (_st, [_vp, _i64, _i64, _i32, _dbl, _i32, _ctx_pp]),
    "gkl_create_ex": (_st, [_vp, _i64, _i64, _i32, _dbl, _i32, ctypes.POINTER(gkl_options),
                            _ctx_pp]),
    "gkl_solve": (_st, [_vp, _vp, _vp, _i64, _vp, _i64, ctypes.POINTER(gkl_info)]),
    "gkl_destroy": (None, [_vp]),
    "gkl_create_batched": (_st, [_i32, _vp, _vp, _vp, _i32, _dbl, _i32,
                                 ctypes.POINTER(gkl_options), _ctx_pp]),
    "gkl_solve_batched": (_st, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gkl_create_loco": (_st, [_vp, _i64, _i64, _i32, _vp, _i32, _dbl, ctypes.POINTER(gkl_options),
                              _ctx_pp]),
    "gkl_batched_plan": (_st, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gkl_column_stats": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "gkl_unpack": (_st, [_vp, _vp]),
    "gkl_matvec": (_st, [_vp, _vp, _vp]),
    "gkl_rmatvec": (_st, [_vp, _vp, _vp]),
    "gkl_matmat_mixed": (_st, [_vp, _vp, _i32, _vp]),
    "gkl_rmatmat_mixed": (_st, [_vp, _vp, _i32, _vp]),
    "gkl_get_trace": (_st, [_vp, _vp, _i64, ctypes.POINTER(_i64)]),
    "gkl_dense_svd": (_st, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "gkl_dense_svd_noalloc": (_st, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "gkl_read_rate": (_st, [_vp, _i64, _i32, _vp, ctypes.POINTER(_dbl)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def declared_functions():
    """Function names declared in include/gkl.h (used by the ABI export test)."""
    with open(_HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gkl_[a-z_]+)\s*\(", text)))


# ---------------------------------------------------------------------------
# thin wrappers (same names as the C ABI)
# ---------------------------------------------------------------------------

def _ptr(x):
    """Device pointer of a torch tensor, or an int / None passed through."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def gkl_options_default():
    o = gkl_options()
    lib.gkl_options_default(ctypes.byref(o))
    return o


def gkl_status_string(s):
    return lib.gkl_status_string(int(s)).decode()


def gkl_last_error(ctx=None):
    return lib.gkl_last_error(ctx).decode()


def _check(status, ctx=None, allow=()):
    if status != GKL_OK and status not in allow:
        raise GKLError(status, gkl_last_error(ctx))
    return status


def gkl_create(G, n, p, k, tol, reorth):
    ctx = ctypes.c_void_p()
    _check(lib.gkl_create(_ptr(G), n, p, k, tol, reorth, ctypes.byref(ctx)))
    return ctx.value


def gkl_create_ex(G, n, p, k, tol, reorth, opt):
    ctx = ctypes.c_void_p()
    _check(lib.gkl_create_ex(_ptr(G), n, p, k, tol, reorth, ctypes.byref(opt), ctypes.byref(ctx)))
    return ctx.value


def gkl_solve(ctx, sigma, U, ldu, V, ldv, allow_not_converged=True):
    info = gkl_info()
    st = lib.gkl_solve(ctx, _ptr(sigma), _ptr(U), ldu, _ptr(V), ldv, ctypes.byref(info))
    _check(st, ctx, allow=(GKL_NOT_CONVERGED,) if allow_not_converged else ())
    return st, info


def gkl_destroy(ctx):
    lib.gkl_destroy(ctx)


def gkl_create_batched(Gs, ns, ps, k, tol, reorth, opt):
    count = len(Gs)
    GA = (ctypes.c_void_p * count)(*[_ptr(g) for g in Gs])
    NA = (ctypes.c_int64 * count)(*ns)
    PA = (ctypes.c_int64 * count)(*ps)
    ctx = ctypes.c_void_p()
    _check(lib.gkl_create_batched(count, GA, NA, PA, k, tol, reorth, ctypes.byref(opt),
                                  ctypes.byref(ctx)))
    return ctx.value


def gkl_create_loco(G, n, p, block_start, k, tol, opt):
    nb = len(block_start) - 1
    BS = (ctypes.c_int64 * (nb + 1))(*[int(x) for x in block_start])
    ctx = ctypes.c_void_p()
    _check(lib.gkl_create_loco(_ptr(G), n, p, nb, BS, k, tol, ctypes.byref(opt), ctypes.byref(ctx)))
    return ctx.value


def gkl_solve_batched(ctx, sigmas, Us, ldus, Vs, ldvs):
    count = len(sigmas)
    SA = (ctypes.c_void_p * count)(*[_ptr(x) for x in sigmas])
    UA = (ctypes.c_void_p * count)(*[_ptr(x) for x in Us])
    LU = (ctypes.c_int64 * count)(*ldus)
    VA = (ctypes.c_void_p * count)(*[_ptr(x) for x in Vs])
    LV = (ctypes.c_int64 * count)(*ldvs)
    infos = (gkl_info * count)()
    st = lib.gkl_solve_batched(ctx, SA, UA, LU, VA, LV, infos)
    _check(st, ctx, allow=(GKL_NOT_CONVERGED,))
    return st, list(infos)


def gkl_batched_plan(ctx):
    mt, rt = ctypes.c_int64(), ctypes.c_int64()
    gm, gr = ctypes.c_int32(), ctypes.c_int32()
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib.gkl_batched_plan(ctx, ctypes.byref(mt), ctypes.byref(rt), ctypes.byref(gm),
                                ctypes.byref(gr), ctypes.byref(a), ctypes.byref(b)), ctx)
    return {"mv_target": mt.value, "rmv_target": rt.value, "grid_mv": gm.value,
            "grid_rmv": gr.value, "mv_ms": a.value, "rmv_ms": b.value}


def gkl_column_stats(ctx, count, nobs, mean, inv_sd):
    _check(lib.gkl_column_stats(ctx, _ptr(count), _ptr(nobs), _ptr(mean), _ptr(inv_sd)), ctx)


def gkl_unpack(ctx, out):
    _check(lib.gkl_unpack(ctx, _ptr(out)), ctx)


def gkl_matvec(ctx, v, y):
    _check(lib.gkl_matvec(ctx, _ptr(v), _ptr(y)), ctx)


def gkl_rmatvec(ctx, u, z):
    _check(lib.gkl_rmatvec(ctx, _ptr(u), _ptr(z)), ctx)


def gkl_matmat_mixed(ctx, W, b, Y):
    _check(lib.gkl_matmat_mixed(ctx, _ptr(W), b, _ptr(Y)), ctx)


def gkl_rmatmat_mixed(ctx, X, b, Z):
    _check(lib.gkl_rmatmat_mixed(ctx, _ptr(X), b, _ptr(Z)), ctx)


def gkl_get_trace(ctx, max_rows=100000):
    import numpy as np
    buf = np.zeros(max_rows * GKL_TRACE_FIELDS)
    written = ctypes.c_int64()
    _check(lib.gkl_get_trace(ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.size,
                             ctypes.byref(written)), ctx)
    return buf[: written.value * GKL_TRACE_FIELDS].reshape(-1, GKL_TRACE_FIELDS)


def gkl_dense_svd(B, m, P, S, Q, stream=None):
    _check(lib.gkl_dense_svd(_ptr(B), m, _ptr(P), _ptr(S), _ptr(Q), stream))


def gkl_dense_svd_noalloc(B, m, P, S, Q, stream=None):
    _check(lib.gkl_dense_svd_noalloc(_ptr(B), m, _ptr(P), _ptr(S), _ptr(Q), stream))


def gkl_read_rate(buf, reps=5, stream=None):
    """Milliseconds of one plain streaming read of the device tensor buf."""
    ms = _dbl(0.0)
    nbytes = buf.numel() * buf.element_size()
    _check(lib.gkl_read_rate(_ptr(buf), nbytes, reps, stream, ctypes.byref(ms)))
    return ms.value


# ---------------------------------------------------------------------------
# convenience: a context object over torch tensors
# ---------------------------------------------------------------------------

class Context:
    """Owns one gkl_ctx; G is a torch.uint8 CUDA tensor of shape (p, ld)."""

    def __init__(self, G, n, p, k, tol=1e-10, reorth=GKL_REORTH_FULL, **options):
        import torch
        self._torch = torch
        self.G = G                      # keep the borrowed matrix alive
        self.n, self.p, self.k = int(n), int(p), int(k)
        opt = gkl_options_default()
        self._v0 = None
        for key, val in options.items():
            if key == "v0":
                if val is not None:
                    self._v0 = val
                    opt.v0 = val.data_ptr()
            elif key == "stream":
                opt.stream = val
            else:
                setattr(opt, key, val)
        if opt.stream is None:
            opt.stream = torch.cuda.current_stream().cuda_stream
        if not opt.ld_bytes:
            opt.ld_bytes = G.shape[1] if G.dim() == 2 else 0
        self.opt = opt
        self.ctx = gkl_create_ex(G, self.n, self.p, self.k, tol, reorth, opt)

    def solve(self, allow_not_converged=True):
        torch = self._torch
        dev = self.G.device
        sigma = torch.empty(self.k, dtype=torch.float64, device=dev)
        U = torch.empty((self.k, self.n), dtype=torch.float64, device=dev)
        V = torch.empty((self.k, self.p), dtype=torch.float64, device=dev)
        st, info = gkl_solve(self.ctx, sigma, U, self.n, V, self.p, allow_not_converged)
        return sigma, U.T, V.T, st, info

    def column_stats(self):
        torch = self._torch
        dev = self.G.device
        out = (torch.empty(self.p, dtype=torch.int64, device=dev),
               torch.empty(self.p, dtype=torch.int64, device=dev),
               torch.empty(self.p, dtype=torch.float64, device=dev),
               torch.empty(self.p, dtype=torch.float64, device=dev))
        gkl_column_stats(self.ctx, *out)
        return out

    def unpack(self):
        out = self._torch.empty((self.p, self.n), dtype=self._torch.int8, device=self.G.device)
        gkl_unpack(self.ctx, out)
        return out.T

    def matvec(self, v):
        y = self._torch.empty(self.n, dtype=self._torch.float64, device=self.G.device)
        gkl_matvec(self.ctx, v.contiguous(), y)
        return y

    def rmatvec(self, u):
        z = self._torch.empty(self.p, dtype=self._torch.float64, device=self.G.device)
        gkl_rmatvec(self.ctx, u.contiguous(), z)
        return z

    def matmat_mixed(self, W):
        """W: (p, b) float64 -> (n, b)."""
        b = W.shape[1]
        Wc = W.T.contiguous()            # column-major p x b
        Y = self._torch.empty((b, self.n), dtype=self._torch.float64, device=self.G.device)
        gkl_matmat_mixed(self.ctx, Wc, b, Y)
        return Y.T

    def rmatmat_mixed(self, X):
        b = X.shape[1]
        Xc = X.T.contiguous()
        Z = self._torch.empty((b, self.p), dtype=self._torch.float64, device=self.G.device)
        gkl_rmatmat_mixed(self.ctx, Xc, b, Z)
        return Z.T

    def trace(self):
        return gkl_get_trace(self.ctx)

    def close(self):
        if self.ctx:
            gkl_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedContext:
    """Owns one batched gkl_ctx over a list of torch.uint8 CUDA tensors (p_q, ld_q)."""

    def __init__(self, Gs, ns, ps, k, tol=1e-10, reorth=GKL_REORTH_FULL, **options):
        import torch
        self._torch = torch
        self.Gs = list(Gs)
        self.ns = [int(x) for x in ns]
        self.ps = [int(x) for x in ps]
        self.k = int(k)
        opt = gkl_options_default()
        self._v0 = None
        for key, val in options.items():
            if key == "v0":
                if val is not None:
                    self._v0 = val
                    opt.v0 = val.data_ptr()
            elif key == "stream":
                opt.stream = val
            else:
                setattr(opt, key, val)
        self.opt = opt
        self.ctx = gkl_create_batched(self.Gs, self.ns, self.ps, self.k, tol, reorth, opt)

    def solve(self):
        """Returns (sigmas, Us, Vs, status, infos) as lists over the problems."""
        torch = self._torch
        dev = self.Gs[0].device
        sig = [torch.empty(self.k, dtype=torch.float64, device=dev) for _ in self.ns]
        Us = [torch.empty((self.k, n), dtype=torch.float64, device=dev) for n in self.ns]
        Vs = [torch.empty((self.k, p), dtype=torch.float64, device=dev) for p in self.ps]
        st, infos = gkl_solve_batched(self.ctx, sig, Us, self.ns, Vs, self.ps)
        return sig, [u.T for u in Us], [v.T for v in Vs], st, infos

    def plan(self):
        return gkl_batched_plan(self.ctx)

    def close(self):
        if self.ctx:
            gkl_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(G, n, p, k, tol=1e-10, reorth=GKL_REORTH_FULL, **options):
    """One-shot top-k solve; returns (sigma, U, V, status, info)."""
    ctx = Context(G, n, p, k, tol, reorth, **options)
    try:
        return ctx.solve()
    finally:
        ctx.close()


class LocoContext(BatchedContext):
    """Leave-one-block-out PCAs over one torch.uint8 CUDA tensor G (p, ld) with
    SNP blocks [block_start[q], block_start[q+1]); solve() returns per-problem
    lists like BatchedContext (V of problem q is p x k, zero on block q)."""

    def __init__(self, G, n, p, block_start, k, tol=1e-8, **options):
        import torch
        self._torch = torch
        self.Gs = [G]
        nb = len(block_start) - 1
        self.ns = [int(n)] * nb
        self.ps = [int(p)] * nb
        self.k = int(k)
        opt = gkl_options_default()
        self._v0 = None
        for key, val in options.items():
            if key == "v0":
                if val is not None:
                    self._v0 = val
                    opt.v0 = val.data_ptr()
            elif key == "stream":
                opt.stream = val
            else:
                setattr(opt, key, val)
        if not opt.ld_bytes:
            opt.ld_bytes = G.shape[1] if G.dim() == 2 else 0
        self.opt = opt
        self.ctx = gkl_create_loco(G, int(n), int(p), list(block_start), self.k, tol, opt)
