"""Plain FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library:
the arithmetic lives in ``orc.c`` (plain C, double precision, one thread,
ascending loops) and this module only marshals numpy arrays through ctypes.

Array conventions follow the paper's element-array view (Section 1, Fig. 2):
``coords (n_nodes, dim)``, ``elems (n_elems, nb)``, local matrices
``(n_elems, nb, nb)``; vectors are float64 of length n_nodes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import build_oracle, library_path

__all__ = [
    "lib",
    "local_matrices",
    "rhs",
    "rhs_local",
    "residual",
    "residual_alg1",
    "residual_scale",
    "jacobi_diag",
    "pcg",
    "richardson",
    "cheb2",
    "cheb3",
    "cheb3_listing",
    "mask_from_nodes",
    "OracleError",
]


class OracleError(RuntimeError):
    pass


_LIB = None

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_I64 = ctypes.c_int64


def lib():
    """Load liborc.so, compiling it first if it has never been built."""
    global _LIB
    if _LIB is None:
        path = os.environ.get("ORACLE_LIB") or library_path()
        if not os.path.exists(path):
            build_oracle()
        L = ctypes.CDLL(path)
        L.orc_local_matrices.argtypes = [ctypes.c_int, _I64, _I64, _D, _I32, _D, _D, _D]
        L.orc_rhs.argtypes = [ctypes.c_int, _I64, _I64, _I32, _D, _D, _D]
        L.orc_rhs_local.argtypes = [ctypes.c_int, _I64, _I64, _I32, _D, _D, _D]
        L.orc_residual_alg1.argtypes = [ctypes.c_int, _I64, _I64, _I32, _D, _D, ctypes.c_double, _D, _D, _D]
        L.orc_residual.argtypes = [ctypes.c_int, _I64, _I64, _I32, _D, _D, ctypes.c_double, _D, _D, _U8, _D]
        L.orc_residual_scale.argtypes = [ctypes.c_int, _I64, _I64, _I32, _D, _D, ctypes.c_double, _D, _D, _D]
        L.orc_jacobi_diag.argtypes = [ctypes.c_int, _I64, _I64, _I32, _D, _D, ctypes.c_double, _D]
        L.orc_pcg.argtypes = [ctypes.c_int, _I64, _I64, _I32, _D, _D, ctypes.c_double, _D, _U8,
                              ctypes.c_int, ctypes.c_double, ctypes.c_int, _D, _D, _D, _D]
        for name in ("orc_richardson", "orc_cheb3", "orc_cheb3_listing"):
            getattr(L, name).argtypes = [ctypes.c_int, _I64, _I64, _I32, _D, _D, ctypes.c_double, _D, _U8,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, _D]
        L.orc_cheb2.argtypes = [ctypes.c_int, _I64, _I64, _I32, _D, _D, ctypes.c_double, _D, _U8,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, _D]
        for fn in (L.orc_local_matrices, L.orc_rhs, L.orc_rhs_local, L.orc_residual_alg1, L.orc_residual,
                   L.orc_residual_scale, L.orc_jacobi_diag, L.orc_pcg, L.orc_richardson, L.orc_cheb2,
                   L.orc_cheb3, L.orc_cheb3_listing):
            fn.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _i(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I32)


def _u8(a):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(_U8)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def mask_from_nodes(n_nodes: int, nodes) -> np.ndarray:
    m = np.zeros(n_nodes, dtype=np.uint8)
    if nodes is not None and len(nodes):
        m[np.asarray(nodes, dtype=np.int64)] = 1
    return m


def _elems(elems):
    return np.ascontiguousarray(elems, dtype=np.int32)


def local_matrices(coords, elems):
    """K_e, M_e (n_elems, nb, nb) and vol (n_elems,) by the P1 formulas."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    elems = _elems(elems)
    dim = coords.shape[1]
    ne, nb = elems.shape
    K = np.empty((ne, nb, nb))
    M = np.empty((ne, nb, nb))
    vol = np.empty(ne)
    _check(lib().orc_local_matrices(dim, coords.shape[0], ne, _d(coords), _i(elems), _d(K), _d(M), _d(vol)),
           "orc_local_matrices")
    return K, M, vol


def rhs(n_nodes, elems, M, f):
    elems = _elems(elems)
    ne, nb = elems.shape
    b = np.empty(n_nodes)
    _check(lib().orc_rhs(nb, n_nodes, ne, _i(elems), _d(_f64(M)), _d(_f64(f)), _d(b)), "orc_rhs")
    return b


def rhs_local(n_nodes, elems, M, f):
    elems = _elems(elems)
    ne, nb = elems.shape
    be = np.empty((ne, nb))
    _check(lib().orc_rhs_local(nb, n_nodes, ne, _i(elems), _d(_f64(M)), _d(_f64(f)), _d(be)), "orc_rhs_local")
    return be


def residual_alg1(n_nodes, elems, K, M, nu, be, x):
    elems = _elems(elems)
    ne, nb = elems.shape
    r = np.empty(n_nodes)
    _check(lib().orc_residual_alg1(nb, n_nodes, ne, _i(elems), _d(_f64(K)), _d(_f64(M)), float(nu),
                                   _d(_f64(be)), _d(_f64(x)), _d(r)), "orc_residual_alg1")
    return r


def residual(n_nodes, elems, K, M, nu, b, x, mask=None):
    elems = _elems(elems)
    ne, nb = elems.shape
    r = np.empty(n_nodes)
    _check(lib().orc_residual(nb, n_nodes, ne, _i(elems), _d(_f64(K)), _d(_f64(M)), float(nu), _d(_f64(b)),
                              _d(_f64(x)), _u8(mask), _d(r)), "orc_residual")
    return r


def residual_scale(n_nodes, elems, K, M, nu, b, x):
    elems = _elems(elems)
    ne, nb = elems.shape
    s = np.empty(n_nodes)
    _check(lib().orc_residual_scale(nb, n_nodes, ne, _i(elems), _d(_f64(K)), _d(_f64(M)), float(nu),
                                    _d(_f64(b)), _d(_f64(x)), _d(s)), "orc_residual_scale")
    return s


def jacobi_diag(n_nodes, elems, K, M, nu):
    elems = _elems(elems)
    ne, nb = elems.shape
    d = np.empty(n_nodes)
    _check(lib().orc_jacobi_diag(nb, n_nodes, ne, _i(elems), _d(_f64(K)), _d(_f64(M)), float(nu), _d(d)),
           "orc_jacobi_diag")
    return d


def pcg(n_nodes, elems, K, M, nu, b, mask, x0, rtol=1e-8, max_iter=10000, jacobi=True, history=False,
        raise_on_noconv=True):
    """Jacobi-PCG.  Returns (x, info) with info = dict(iters, relres, r0, replacements, status)."""
    elems = _elems(elems)
    ne, nb = elems.shape
    x = np.array(x0, dtype=np.float64, copy=True)
    out = np.zeros(4)
    ah = np.zeros(max_iter) if history else None
    bh = np.zeros(max_iter) if history else None
    rc = lib().orc_pcg(nb, n_nodes, ne, _i(elems), _d(_f64(K)), _d(_f64(M)), float(nu), _d(_f64(b)), _u8(mask),
                       1 if jacobi else 0, float(rtol), int(max_iter), _d(x), _d(out), _d(ah), _d(bh))
    if rc not in (0, -3) or (rc == -3 and raise_on_noconv):
        _check(rc, "orc_pcg")
    info = dict(iters=int(out[0]), relres=float(out[1]), r0=float(out[2]), replacements=int(out[3]), status=rc)
    if history:
        info["alpha"] = ah[: info["iters"]]
        info["beta"] = bh[: max(info["iters"] - 1, 0)]
    return x, info


def _iter(fn, n_nodes, elems, K, M, nu, b, mask, x0, *args):
    elems = _elems(elems)
    ne, nb = elems.shape
    x = np.array(x0, dtype=np.float64, copy=True)
    _check(fn(nb, n_nodes, ne, _i(elems), _d(_f64(K)), _d(_f64(M)), float(nu), _d(_f64(b)), _u8(mask), *args,
              _d(x)), fn.__name__)
    return x


def richardson(n_nodes, elems, K, M, nu, b, mask, x0, lam1, lam2, iters):
    return _iter(lib().orc_richardson, n_nodes, elems, K, M, nu, b, mask, x0, float(lam1), float(lam2), int(iters))


def cheb2(n_nodes, elems, K, M, nu, b, mask, x0, lam1, lam2, N, iters):
    return _iter(lib().orc_cheb2, n_nodes, elems, K, M, nu, b, mask, x0, float(lam1), float(lam2), int(N),
                 int(iters))


def cheb3(n_nodes, elems, K, M, nu, b, mask, x0, lam1, lam2, iters):
    return _iter(lib().orc_cheb3, n_nodes, elems, K, M, nu, b, mask, x0, float(lam1), float(lam2), int(iters))


def cheb3_listing(n_nodes, elems, K, M, nu, b, mask, x0, lam1, lam2, iters):
    return _iter(lib().orc_cheb3_listing, n_nodes, elems, K, M, nu, b, mask, x0, float(lam1), float(lam2),
                 int(iters))
