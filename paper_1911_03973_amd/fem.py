"""Thin ctypes binding of libfem.so (the C ABI of include/fem.h).

Only argument marshalling lives here: torch tensors provide device memory and
the current HIP stream, every computation runs in the library's HIP kernels.
Importing this module loads the library and raises ``ImportError`` if it has
not been built (``python paper_1911_03973_amd/build.py``) -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libfem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libfem.so is not built ({LIB_PATH}); run paper_1911_03973_amd/build.py")

_lib = ctypes.CDLL(LIB_PATH)

FEM_OK, FEM_EINVAL, FEM_EHIP, FEM_ENOCONV, FEM_ESINGULAR, FEM_EBREAKDOWN, FEM_ENOMEM = 0, -1, -2, -3, -4, -5, -6
F64, F32, F32X2 = 0, 1, 2
MFREE = 3  # matrix-free: K_e, M_e rebuilt from the coordinates in every pass
PRECOND_NONE, PRECOND_JACOBI = 0, 1
SMOOTH_JACOBI, SMOOTH_CHEBYSHEV = 0, 1  # multigrid smoothers
LOSS_L2, LOSS_ENERGY = 0, 1  # U-Net training losses

_STATUS = {
    FEM_EINVAL: "FEM_EINVAL",
    FEM_EHIP: "FEM_EHIP",
    FEM_ENOCONV: "FEM_ENOCONV",
    FEM_ESINGULAR: "FEM_ESINGULAR",
    FEM_EBREAKDOWN: "FEM_EBREAKDOWN",
    FEM_ENOMEM: "FEM_ENOMEM",
}


class FemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class PlanStats(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n_b", ctypes.c_int),
        ("n_nodes", ctypes.c_int64), ("n_elems", ctypes.c_int64), ("n_dirichlet", ctypes.c_int64),
        ("chunk_elems", ctypes.c_int), ("n_chunks", ctypes.c_int64), ("n_local", ctypes.c_int64),
        ("n_shared", ctypes.c_int64), ("n_partials", ctypes.c_int64), ("index_bytes", ctypes.c_int64),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int), ("nu", ctypes.c_double), ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int),
        ("precond", ctypes.c_int), ("inner_rtol", ctypes.c_double), ("max_outer", ctypes.c_int),
        ("check_every", ctypes.c_int), ("profile", ctypes.c_int), ("vectors", ctypes.c_int),
        ("block", ctypes.c_int),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("iters", ctypes.c_int), ("outer", ctypes.c_int), ("replacements", ctypes.c_int),
        ("relres", ctypes.c_double), ("r0", ctypes.c_double), ("seconds", ctypes.c_double),
        ("matvec_ms", ctypes.c_double), ("matvec_samples", ctypes.c_int), ("matvec_calls", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchOpts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int), ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int), ("refresh", ctypes.c_double),
        ("max_refresh", ctypes.c_int), ("block", ctypes.c_int), ("grid", ctypes.c_int),
        ("watchdog_seconds", ctypes.c_double), ("use_graph", ctypes.c_int), ("group", ctypes.c_int),
        ("items_per_phase", ctypes.c_int), ("inline_segments", ctypes.c_int), ("adaptive", ctypes.c_int),
    ]


class BatchResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("iters", ctypes.c_int), ("refreshes", ctypes.c_int), ("relres", ctypes.c_double),
        ("r0", ctypes.c_double),
    ]


class FcgOpts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int), ("nu", ctypes.c_double), ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int),
        ("grid_n", ctypes.c_int), ("cval", ctypes.c_double), ("stall_iters", ctypes.c_int),
        ("max_replace", ctypes.c_int), ("smooth", ctypes.c_int), ("omega", ctypes.c_double),
        ("graph", ctypes.c_int), ("check_every", ctypes.c_int), ("cycle_dtype", ctypes.c_int),
    ]


class FcgInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("iters", ctypes.c_int), ("pcg_iters", ctypes.c_int),
        ("precond_calls", ctypes.c_int), ("fell_back", ctypes.c_int), ("fallback_reason", ctypes.c_int),
        ("replacements", ctypes.c_int), ("relres", ctypes.c_double), ("r0", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]


class IterOpts(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int), ("dtype", ctypes.c_int), ("nu", ctypes.c_double), ("lam1", ctypes.c_double),
        ("lam2", ctypes.c_double), ("cycle", ctypes.c_int), ("iters", ctypes.c_int),
    ]


class IterInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("iters", ctypes.c_int), ("relres", ctypes.c_double), ("r0", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]


RICHARDSON, CHEBYSHEV2, CHEBYSHEV3, CHEBYSHEV3_LISTING = 0, 1, 2, 3


class MgOpts(ctypes.Structure):
    _fields_ = [
        ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int), ("smooth", ctypes.c_int), ("omega", ctypes.c_double),
        ("max_replace", ctypes.c_int), ("cycle_dtype", ctypes.c_int), ("smoother", ctypes.c_int),
        ("cheb_lower", ctypes.c_double),
    ]


_vp, _i64, _int, _dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
_SIGS = {
    "fem_plan_create": [_int, _i64, _i64, _vp, _vp, _vp, _i64, _int, _vp, ctypes.POINTER(_vp)],
    "fem_plan_create_p2": [_int, _i64, _i64, _vp, _vp, _vp, _i64, _int, _vp, ctypes.POINTER(_vp)],
    "fem_plan_destroy": [_vp],
    "fem_plan_check_host": [_int, _i64, _i64, _vp, _vp, _vp, _i64, _int, ctypes.POINTER(PlanStats)],
    "fem_plan_check_host_p2": [_int, _i64, _i64, _vp, _vp, _vp, _i64, _int, ctypes.POINTER(PlanStats)],
    "fem_plan_get_stats": [_vp, ctypes.POINTER(PlanStats)],
    "fem_build_local_matrices": [_vp, _int, _vp, _vp, _vp, _vp],
    "fem_combine_local": [_vp, _int, _vp, _vp, _dbl, _int, _vp, _vp],
    "fem_element_residual": [_vp, _int, _vp, _vp, _dbl, _vp, _vp, _vp, _int, _vp],
    "fem_element_residual_f32": [_vp, _vp, _vp, _vp, _vp, _int, _vp],
    "fem_element_residual_noalloc": [_vp, _int, _vp, _vp, _dbl, _vp, _vp, _vp, _int, _vp],
    "fem_jacobi_diag": [_vp, _int, _vp, _vp, _dbl, _vp, _vp],
    "fem_assemble_rhs": [_vp, _int, _vp, _vp, _vp, _vp],
    "fem_pcg_solve": [_vp, ctypes.POINTER(SolveOpts), _vp, _vp, _vp, _vp, ctypes.POINTER(SolveInfo), _vp],
    "fem_batch_create": [_int, _int, _vp, _vp, _vp, _vp, _vp, _vp, _int, _vp, ctypes.POINTER(_vp)],
    "fem_batch_destroy": [_vp],
    "fem_batch_get_stats": [_vp, ctypes.POINTER(PlanStats)],
    "fem_batch_build_local_matrices": [_vp, _int, _vp, _vp, _vp],
    "fem_batch_assemble_rhs": [_vp, _int, _vp, _vp, _vp, _vp],
    "fem_batch_solve": [_vp, ctypes.POINTER(BatchOpts), _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(BatchResult),
                        ctypes.POINTER(ctypes.c_double), _vp],
    "fem_unet_create": [_int, _int, _int, _int, ctypes.c_uint64, _vp, ctypes.POINTER(_vp)],
    "fem_unet_destroy": [_vp],
    "fem_unet_param_count": [_vp, ctypes.POINTER(_i64)],
    "fem_unet_get_params": [_vp, _vp, _vp],
    "fem_unet_set_params": [_vp, _vp, _vp],
    "fem_unet_forward": [_vp, _int, _vp, _vp, _vp],
    "fem_unet_loss_grad": [_vp, _int, _vp, _vp, _vp, _vp, _vp],
    "fem_unet_train_step": [_vp, _int, _vp, _vp, ctypes.c_float, _vp, _vp],
    "fem_unet_set_loss": [_vp, _int, ctypes.c_double],
    "fem_unet_set_output_smoothing": [_vp, _int],
    "fem_unet_precondition": [_vp, _int, _vp, _dbl, _vp, _vp, _vp],
    "fem_unet_make_pair": [_vp, _int, _vp, _vp, _vp, _dbl, _vp, _vp, _vp],
    "fem_fcg_solve": [_vp, ctypes.POINTER(FcgOpts), _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(FcgInfo), _vp],
    "fem_fcg_precondition": [_vp, ctypes.POINTER(FcgOpts), _vp, _vp, _vp, _vp, _vp, _vp],
    "fem_iterate": [_vp, ctypes.POINTER(IterOpts), _vp, _vp, _vp, _vp, ctypes.POINTER(IterInfo), _vp],
    "fem_mg_create": [_int, _vp, _vp, _int, _vp, _vp, _dbl, _vp, ctypes.POINTER(_vp)],
    "fem_mg_destroy": [_vp],
    "fem_mg_solve": [_vp, ctypes.POINTER(MgOpts), _vp, _vp, ctypes.POINTER(FcgInfo), _vp],
    "fem_mg_galerkin_apply": [_vp, _int, _vp, _vp, _vp],
    "fem_mg_vcycle": [_vp, ctypes.POINTER(MgOpts), _vp, _vp, _vp],
    "fem_mg_level_bound": [_vp, _int, ctypes.POINTER(_dbl)],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.fem_last_error.restype = ctypes.c_char_p
_lib.fem_last_error.argtypes = []
_lib.fem_solve_opts_default.argtypes = [ctypes.POINTER(SolveOpts)]
_lib.fem_solve_opts_default.restype = None
_lib.fem_batch_opts_default.argtypes = [ctypes.POINTER(BatchOpts)]
_lib.fem_batch_opts_default.restype = None
_lib.fem_fcg_opts_default.argtypes = [ctypes.POINTER(FcgOpts)]
_lib.fem_fcg_opts_default.restype = None
_lib.fem_iter_opts_default.argtypes = [ctypes.POINTER(IterOpts)]
_lib.fem_iter_opts_default.restype = None
_lib.fem_mg_opts_default.argtypes = [ctypes.POINTER(MgOpts)]
_lib.fem_mg_opts_default.restype = None

EXPORTED = sorted(list(_SIGS) + ["fem_last_error", "fem_solve_opts_default", "fem_batch_opts_default",
                                 "fem_fcg_opts_default", "fem_iter_opts_default", "fem_mg_opts_default"])


def library():
    return _lib


def _check(rc, allow=()):
    if rc != FEM_OK and rc not in allow:
        raise FemError(rc, _lib.fem_last_error().decode())
    return rc


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, numel, what):
    if t is None:
        return
    if t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {t.numel()}")


def matrix_shape(dtype, nb, n_elems):
    """Tensor shape and torch dtype of one local-matrix array in `dtype` storage."""
    if dtype == F64:
        return (nb * nb, n_elems), torch.float64
    if dtype == F32:
        return (nb * nb, n_elems), torch.float32
    if dtype == F32X2:
        return (2, nb * nb, n_elems), torch.float32
    raise ValueError("unknown dtype")


class Plan:
    """Owns a fem_plan (chunked element -> node index of one mesh)."""

    def __init__(self, dim, coords_soa, conn_soa, dirichlet=None, chunk_elems=0, stream=None):
        """conn_soa (n_b, n_elems): n_b = dim + 1, or 6 / 10 for quadratic triangles / tetrahedra."""
        n_nodes = coords_soa.shape[1]
        n_elems = conn_soa.shape[1]
        nb = int(conn_soa.shape[0])
        if nb != dim + 1 and (dim, nb) not in ((2, 6), (3, 10)):
            raise ValueError("conn must list dim + 1 nodes (linear) or 6 / 10 nodes (quadratic triangles / "
                             "tetrahedra) per element")
        _need(coords_soa, torch.float64, dim * n_nodes, "coords")
        _need(conn_soa, torch.int32, nb * n_elems, "conn")
        if dirichlet is not None and dirichlet.numel() == 0:
            dirichlet = None
        if dirichlet is not None:
            _need(dirichlet, torch.int32, dirichlet.numel(), "dirichlet")
        h = ctypes.c_void_p()
        nd = 0 if dirichlet is None else dirichlet.numel()
        cp = _ptr(conn_soa) if n_elems else None
        if nb > dim + 1:
            _check(_lib.fem_plan_create_p2(dim, n_nodes, n_elems, _ptr(coords_soa), cp, _ptr(dirichlet), nd, chunk_elems,
                                           _stream(stream), ctypes.byref(h)))
        else:
            _check(_lib.fem_plan_create(dim, n_nodes, n_elems, _ptr(coords_soa), cp, _ptr(dirichlet), nd, chunk_elems,
                                        _stream(stream), ctypes.byref(h)))
        self._h = h
        self.dim, self.nb, self.n_nodes, self.n_elems = dim, nb, n_nodes, n_elems
        self.device = coords_soa.device

    @classmethod
    def from_mesh(cls, mesh, dirichlet=None, chunk_elems=0, device="cuda"):
        coords = torch.from_numpy(mesh.coords.T.copy()).to(device)
        conn = torch.from_numpy(mesh.elems.T.copy()).to(device)
        d = None if dirichlet is None else torch.as_tensor(dirichlet, dtype=torch.int32).to(device)
        return cls(mesh.dim, coords.contiguous(), conn.contiguous(), d, chunk_elems)

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("plan destroyed")
        return self._h

    def stats(self):
        st = PlanStats()
        _check(_lib.fem_plan_get_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def destroy(self):
        if getattr(self, "_h", None):
            _lib.fem_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def empty_matrix(self, dtype):
        shape, tdt = matrix_shape(dtype, self.nb, self.n_elems)
        return torch.empty(shape, dtype=tdt, device=self.device)

    def empty_vector(self, tdt=torch.float64):
        return torch.empty(self.n_nodes, dtype=tdt, device=self.device)

    def _mat(self, t, dtype, what):
        if t is None or dtype == MFREE:
            return
        shape, tdt = matrix_shape(dtype, self.nb, self.n_elems)
        _need(t, tdt, int(torch.Size(shape).numel()), what)


def plan_check_host(mesh, dirichlet=None, chunk_elems=0):
    """Host-only validation and sizing of a plan (no GPU needed).  Returns the stats dict."""
    import numpy as np

    coords = np.ascontiguousarray(mesh.coords.T, dtype=np.float64)
    conn = np.ascontiguousarray(mesh.elems.T, dtype=np.int32)
    d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.int32)
    st = PlanStats()
    fn = _lib.fem_plan_check_host_p2 if conn.shape[0] > mesh.dim + 1 else _lib.fem_plan_check_host
    _check(fn(mesh.dim, coords.shape[1], conn.shape[1], coords.ctypes.data,
                                    conn.ctypes.data if conn.size else None,
                                    None if d is None or d.size == 0 else d.ctypes.data,
                                    0 if d is None else d.size, chunk_elems, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in st._fields_}


def build_local_matrices(plan, dtype, K=None, M=None, vol=None, stream=None):
    plan._mat(K, dtype, "K_e")
    plan._mat(M, dtype, "M_e")
    _need(vol, torch.float64, plan.n_elems, "vol")
    _check(_lib.fem_build_local_matrices(plan.handle, dtype, _ptr(K), _ptr(M), _ptr(vol), _stream(stream)))


def combine_local(plan, dtype_in, K, M, nu, dtype_out, A, stream=None):
    plan._mat(K, dtype_in, "K_e")
    plan._mat(M, dtype_in, "M_e")
    plan._mat(A, dtype_out, "A_e")
    _check(_lib.fem_combine_local(plan.handle, dtype_in, _ptr(K), _ptr(M), float(nu), dtype_out, _ptr(A),
                                  _stream(stream)))


def element_residual(plan, dtype, K, M, nu, b, x, r, mask=True, stream=None):
    plan._mat(K, dtype, "K_e")
    plan._mat(M, dtype, "M_e")
    for t, w in ((b, "b"), (x, "x"), (r, "r")):
        _need(t, torch.float64, plan.n_nodes, w)
    _check(_lib.fem_element_residual(plan.handle, dtype, _ptr(K), _ptr(M), float(nu), _ptr(b), _ptr(x), _ptr(r),
                                     1 if mask else 0, _stream(stream)))


def element_residual_noalloc(plan, dtype, K, M, nu, b, x, r, mask=True, stream=None):
    """fem_element_residual_noalloc: element_residual with the library's static scratch (allocates nothing)."""
    plan._mat(K, dtype, "K_e")
    plan._mat(M, dtype, "M_e")
    for t, w in ((b, "b"), (x, "x"), (r, "r")):
        _need(t, torch.float64, plan.n_nodes, w)
    _check(_lib.fem_element_residual_noalloc(plan.handle, dtype, _ptr(K), _ptr(M), float(nu), _ptr(b), _ptr(x),
                                             _ptr(r), 1 if mask else 0, _stream(stream)))


def element_residual_f32(plan, A, b, x, r, mask=True, stream=None):
    plan._mat(A, F32, "A_e")
    for t, w in ((b, "b"), (x, "x"), (r, "r")):
        _need(t, torch.float32, plan.n_nodes, w)
    _check(_lib.fem_element_residual_f32(plan.handle, _ptr(A), _ptr(b), _ptr(x), _ptr(r), 1 if mask else 0,
                                         _stream(stream)))


def jacobi_diag(plan, dtype, K, M, nu, d, stream=None):
    plan._mat(K, dtype, "K_e")
    plan._mat(M, dtype, "M_e")
    _need(d, torch.float64, plan.n_nodes, "diag")
    _check(_lib.fem_jacobi_diag(plan.handle, dtype, _ptr(K), _ptr(M), float(nu), _ptr(d), _stream(stream)))


def assemble_rhs(plan, dtype, M, f, b, stream=None):
    plan._mat(M, dtype, "M_e")
    _need(f, torch.float64, plan.n_nodes, "f")
    _need(b, torch.float64, plan.n_nodes, "b")
    _check(_lib.fem_assemble_rhs(plan.handle, dtype, _ptr(M), _ptr(f), _ptr(b), _stream(stream)))


def solve_opts(**kw):
    o = SolveOpts()
    _lib.fem_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def pcg_solve(plan, opts, K, M, b, x, stream=None, allow=(FEM_ENOCONV,)):
    """Runs fem_pcg_solve; returns the info dict (status included)."""
    plan._mat(K, opts.dtype, "K_e")
    plan._mat(M, opts.dtype, "M_e")
    _need(b, torch.float64, plan.n_nodes, "b")
    _need(x, torch.float64, plan.n_nodes, "x")
    info = SolveInfo()
    _check(_lib.fem_pcg_solve(plan.handle, ctypes.byref(opts), _ptr(K), _ptr(M), _ptr(b), _ptr(x),
                              ctypes.byref(info), _stream(stream)), allow=allow)
    return info.as_dict()


def last_error():
    return _lib.fem_last_error().decode()


# ---------------------------------------------------------------------------
# Batches of independent problems
# ---------------------------------------------------------------------------

def batch_opts(**kw):
    o = BatchOpts()
    _lib.fem_batch_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Batch:
    """Owns a fem_batch: independent meshes solved together in one persistent launch."""

    def __init__(self, meshes, dirichlets, chunk_elems=0, device="cuda", stream=None):
        import numpy as np

        dim = meshes[0].dim
        P = len(meshes)
        node_off = np.zeros(P + 1, np.int64)
        elem_off = np.zeros(P + 1, np.int64)
        dir_off = np.zeros(P + 1, np.int64)
        for i, (m, d) in enumerate(zip(meshes, dirichlets)):
            node_off[i + 1] = node_off[i] + m.n_nodes
            elem_off[i + 1] = elem_off[i] + m.n_elems
            dir_off[i + 1] = dir_off[i] + (0 if d is None else len(d))
        coords = np.concatenate([m.coords for m in meshes]).T.copy()
        conn = np.concatenate([m.elems for m in meshes]).T.copy()
        dirs = np.concatenate([np.asarray(d if d is not None else [], np.int32) for d in dirichlets]).astype(np.int32)
        self._coords = torch.from_numpy(coords).to(device)
        self._conn = torch.from_numpy(conn).to(device)
        self._dir = torch.from_numpy(dirs if dirs.size else np.zeros(1, np.int32)).to(device)
        h = ctypes.c_void_p()
        _check(_lib.fem_batch_create(dim, P, node_off.ctypes.data, elem_off.ctypes.data, dir_off.ctypes.data,
                                     _ptr(self._coords), _ptr(self._conn), _ptr(self._dir), chunk_elems,
                                     _stream(stream), ctypes.byref(h)))
        self._h = h
        self.dim, self.nb, self.n_problems = dim, dim + 1, P
        self.node_off, self.elem_off = node_off, elem_off
        self.n_nodes, self.n_elems = int(node_off[-1]), int(elem_off[-1])
        self.device = self._coords.device

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("batch destroyed")
        return self._h

    def destroy(self):
        if getattr(self, "_h", None):
            _lib.fem_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def stats(self):
        st = PlanStats()
        _check(_lib.fem_batch_get_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def empty_matrix(self, dtype):
        shape, tdt = matrix_shape(dtype, self.nb, self.n_elems)
        return torch.empty(shape, dtype=tdt, device=self.device)

    def build_local_matrices(self, dtype, K, M, stream=None):
        _check(_lib.fem_batch_build_local_matrices(self.handle, dtype, _ptr(K), _ptr(M), _stream(stream)))

    def assemble_rhs(self, dtype, M, f, b, stream=None):
        _need(f, torch.float64, self.n_nodes, "f")
        _need(b, torch.float64, self.n_nodes, "b")
        _check(_lib.fem_batch_assemble_rhs(self.handle, dtype, _ptr(M), _ptr(f), _ptr(b), _stream(stream)))

    def solve(self, opts, K, M, nus, b, x, stream=None, allow=(FEM_ENOCONV,)):
        """Returns (status, [per-problem result dicts], seconds)."""
        import numpy as np

        nu = np.ascontiguousarray(nus, dtype=np.float64)
        assert nu.shape == (self.n_problems,)
        _need(b, torch.float64, self.n_nodes, "b")
        _need(x, torch.float64, self.n_nodes, "x")
        res = (BatchResult * self.n_problems)()
        sec = ctypes.c_double(0.0)
        rc = _check(_lib.fem_batch_solve(self.handle, ctypes.byref(opts), _ptr(K), _ptr(M), nu.ctypes.data, _ptr(b),
                                         _ptr(x), res, ctypes.byref(sec), _stream(stream)), allow=allow)
        out = [{k: getattr(r, k) for k, _ in r._fields_} for r in res]
        return rc, out, sec.value


# ---------------------------------------------------------------------------
# Learned preconditioner and flexible CG
# ---------------------------------------------------------------------------

class UNet:
    """Owns a fem_unet: a U-Net on H x W images trained and run by the library's MFMA kernels."""

    def __init__(self, H, W, max_batch=1, channels=16, seed=0, stream=None):
        h = _vp()
        _check(_lib.fem_unet_create(int(H), int(W), int(max_batch), int(channels), int(seed), _stream(stream),
                                    ctypes.byref(h)))
        self._h = h
        self.H, self.W, self.max_batch, self.channels = int(H), int(W), int(max_batch), int(channels)
        cnt = _i64(0)
        _check(_lib.fem_unet_param_count(self._h, ctypes.byref(cnt)))
        self.n_params = cnt.value

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("network destroyed")
        return self._h

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _lib.fem_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def get_params(self, stream=None):
        w = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(_lib.fem_unet_get_params(self.handle, _ptr(w), _stream(stream)))
        return w

    def set_params(self, w, stream=None):
        _need(w, torch.float32, self.n_params, "params")
        _check(_lib.fem_unet_set_params(self.handle, _ptr(w), _stream(stream)))

    def _io(self, inp, target=None):
        B = inp.shape[0]
        _need(inp, torch.float32, B * self.H * self.W * 2, "input")
        if target is not None:
            _need(target, torch.float32, B * self.H * self.W, "target")
        return B

    def forward(self, inp, stream=None):
        """inp float32 [B, H, W, 2] -> float32 [B, H, W]."""
        B = self._io(inp)
        out = torch.empty((B, self.H, self.W), dtype=torch.float32, device="cuda")
        _check(_lib.fem_unet_forward(self.handle, B, _ptr(inp), _ptr(out), _stream(stream)))
        return out

    def set_loss(self, kind, nu_scale=0.0):
        """LOSS_L2, or LOSS_ENERGY with nu = nu_scale * input channel 1 (fem_unet_set_loss)."""
        _check(_lib.fem_unet_set_loss(self.handle, int(kind), float(nu_scale)))

    def set_output_smoothing(self, passes):
        """Binomial smoothing passes after the output layer (fem_unet_set_output_smoothing)."""
        _check(_lib.fem_unet_set_output_smoothing(self.handle, int(passes)))

    def loss_grad(self, inp, target, stream=None):
        """(loss tensor [1] float64, gradient float32 [n_params])."""
        B = self._io(inp, target)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(_lib.fem_unet_loss_grad(self.handle, B, _ptr(inp), _ptr(target), _ptr(loss), _ptr(g),
                                       _stream(stream)))
        return loss, g

    def train_step(self, inp, target, lr, loss=None, stream=None):
        B = self._io(inp, target)
        _check(_lib.fem_unet_train_step(self.handle, B, _ptr(inp), _ptr(target), float(lr), _ptr(loss),
                                        _stream(stream)))

    def precondition(self, grid_n, r, cval, z, mask=None, stream=None):
        n = (grid_n + 1) ** 2
        _need(r, torch.float64, n, "r")
        _need(z, torch.float64, n, "z")
        _need(mask, torch.uint8, n, "mask")
        _check(_lib.fem_unet_precondition(self.handle, int(grid_n), _ptr(r), float(cval), _ptr(mask), _ptr(z),
                                          _stream(stream)))


    def make_pair(self, grid_n, r, u, x, cval, inp, target, stream=None):
        """Writes one training pair through fem_unet_make_pair: inp float32 [grid_n, grid_n, 2]
        (the network input of r), target float32 [grid_n, grid_n] (u - x scaled to unit RMS)."""
        n = (grid_n + 1) ** 2
        for t, name in ((r, "r"), (u, "u"), (x, "x")):
            _need(t, torch.float64, n, name)
        _need(inp, torch.float32, grid_n * grid_n * 2, "input image")
        _need(target, torch.float32, grid_n * grid_n, "target image")
        _check(_lib.fem_unet_make_pair(self.handle, int(grid_n), _ptr(r), _ptr(u), _ptr(x), float(cval), _ptr(inp),
                                       _ptr(target), _stream(stream)))


def fcg_opts(**kw):
    o = FcgOpts()
    _lib.fem_fcg_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def fcg_solve(plan, opts, net, K, M, b, x, stream=None, allow=(FEM_ENOCONV,)):
    """Runs fem_fcg_solve (net None: Jacobi preconditioner); returns the info dict."""
    plan._mat(K, opts.dtype, "K_e")
    plan._mat(M, opts.dtype, "M_e")
    _need(b, torch.float64, plan.n_nodes, "b")
    _need(x, torch.float64, plan.n_nodes, "x")
    info = FcgInfo()
    _check(_lib.fem_fcg_solve(plan.handle, ctypes.byref(opts), net.handle if net is not None else None, _ptr(K),
                              _ptr(M), _ptr(b), _ptr(x), ctypes.byref(info), _stream(stream)), allow=allow)
    return {k: getattr(info, k) for k, _ in info._fields_}


def fcg_precondition(plan, opts, net, K, M, r, z, stream=None):
    """z = B(r) once through fem_fcg_precondition (net None: D^-1 r)."""
    plan._mat(K, opts.dtype, "K_e")
    plan._mat(M, opts.dtype, "M_e")
    _need(r, torch.float64, plan.n_nodes, "r")
    _need(z, torch.float64, plan.n_nodes, "z")
    _check(_lib.fem_fcg_precondition(plan.handle, ctypes.byref(opts), net.handle if net is not None else None,
                                     _ptr(K), _ptr(M), _ptr(r), _ptr(z), _stream(stream)))


# ---------------------------------------------------------------------------
# The paper's iterations (Richardson, 2- and 3-level Chebyshev)
# ---------------------------------------------------------------------------

def iter_opts(**kw):
    o = IterOpts()
    _lib.fem_iter_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def iterate(plan, opts, K, M, b, x, stream=None):
    """Runs fem_iterate (opts.iters steps, x updated in place); returns the info dict."""
    plan._mat(K, opts.dtype, "K_e")
    plan._mat(M, opts.dtype, "M_e")
    _need(b, torch.float64, plan.n_nodes, "b")
    _need(x, torch.float64, plan.n_nodes, "x")
    info = IterInfo()
    _check(_lib.fem_iterate(plan.handle, ctypes.byref(opts), _ptr(K), _ptr(M), _ptr(b), _ptr(x), ctypes.byref(info),
                            _stream(stream)))
    return {k: getattr(info, k) for k, _ in info._fields_}


# ---------------------------------------------------------------------------
# Geometric multigrid on nested square meshes
# ---------------------------------------------------------------------------

def mg_opts(**kw):
    o = MgOpts()
    _lib.fem_mg_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class MG:
    """Owns a fem_mg over plans of nested square meshes (finest first).  Keeps
    references to the plans (which must outlive the hierarchy)."""

    def __init__(self, plans, grid_n, dtype, K, M, nu, stream=None):
        L = len(plans)
        for l in range(L):
            plans[l]._mat(K[l], dtype, "K_e")
            if M is not None and M[l] is not None:
                plans[l]._mat(M[l], dtype, "M_e")
        ph = (_vp * L)(*[p.handle for p in plans])
        gn = (ctypes.c_int * L)(*[int(g) for g in grid_n])
        kh = (_vp * L)(*[_ptr(k) for k in K])
        mh = (_vp * L)(*[(_ptr(m) if m is not None else None) for m in (M if M is not None else [None] * L)])
        h = _vp()
        _check(_lib.fem_mg_create(L, ph, gn, int(dtype), kh, mh, float(nu), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.plans = list(plans)
        self.grid_n = [int(g) for g in grid_n]

    @classmethod
    def from_meshes(cls, meshes, dirichlets, nu, dtype=F64):
        """Plans and local matrices for every level, then the hierarchy."""
        plans, K, M = [], [], []
        for mesh, nd in zip(meshes, dirichlets):
            p = Plan.from_mesh(mesh, nd)
            k = p.empty_matrix(dtype)
            m = p.empty_matrix(dtype)
            build_local_matrices(p, dtype, k, m, None)
            plans.append(p)
            K.append(k)
            M.append(m)
        mg = cls(plans, [m.n for m in meshes], dtype, K, M if nu != 0.0 else None, nu)
        mg.K, mg.M = K, M
        return mg

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("hierarchy destroyed")
        return self._h

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _lib.fem_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def solve(self, opts, b, x, stream=None, allow=(FEM_ENOCONV,)):
        n = self.plans[0].n_nodes
        _need(b, torch.float64, n, "b")
        _need(x, torch.float64, n, "x")
        info = FcgInfo()
        _check(_lib.fem_mg_solve(self.handle, ctypes.byref(opts), _ptr(b), _ptr(x), ctypes.byref(info),
                                 _stream(stream)), allow=allow)
        return {k: getattr(info, k) for k, _ in info._fields_}

    def vcycle(self, r, smooth=2, omega=2.0 / 3.0, z=None, cycle_dtype=F64, stream=None, smoother=SMOOTH_JACOBI,
               cheb_lower=0.3):
        """z = B r, one V-cycle on the finest level."""
        n = self.plans[0].n_nodes
        _need(r, torch.float64, n, "r")
        if z is None:
            z = torch.empty(n, dtype=torch.float64, device="cuda")
        _need(z, torch.float64, n, "z")
        o = mg_opts(smooth=int(smooth), omega=float(omega), cycle_dtype=int(cycle_dtype), smoother=int(smoother),
                    cheb_lower=float(cheb_lower))
        _check(_lib.fem_mg_vcycle(self.handle, ctypes.byref(o), _ptr(r), _ptr(z), _stream(stream)))
        return z

    def level_bound(self, level):
        """Gershgorin bound of D^-1 A on a level (the Chebyshev interval's top)."""
        g = ctypes.c_double()
        _check(_lib.fem_mg_level_bound(self.handle, int(level), ctypes.byref(g)))
        return g.value

    def galerkin_apply(self, level, zc, stream=None):
        _need(zc, torch.float64, self.plans[level + 1].n_nodes, "zc")
        out = torch.empty(self.plans[level + 1].n_nodes, dtype=torch.float64, device="cuda")
        _check(_lib.fem_mg_galerkin_apply(self.handle, int(level), _ptr(zc), _ptr(out), _stream(stream)))
        return out
