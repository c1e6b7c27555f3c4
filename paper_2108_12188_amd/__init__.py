"""Python binding of the MI355X SEM Poisson CG library (libsem.so, C ABI).

Argument marshalling only: every step of the hot path runs in the HIP
kernels behind ``include/sem.h``.  PyTorch provides device memory and the
current HIP stream.  There is no CPU fallback: without the built library
(or without a GPU) every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["SemError", "Mesh", "Batch", "Server", "mesh_footprint", "ax_shape_set",
           "ax_shape_get", "ax_engine_set", "ax_engine_get", "ENGINE_DEFAULT", "ENGINE_VALU",
           "ENGINE_MFMA", "FP64", "FP32", "MIXED", "PRECOMPUTED", "ON_THE_FLY",
           "PRECOND_NONE", "PRECOND_JACOBI", "ORDER_HILBERT", "ORDER_MORTON", "ORDER_ROWS", "element_order",
           "set_cache_bytes",
           "permute_elements", "lib", "library_path", "version"]

FP64, FP32, MIXED = 0, 1, 2
PRECOMPUTED, ON_THE_FLY = 0, 1
PRECOND_NONE, PRECOND_JACOBI = 0, 1
ORDER_HILBERT, ORDER_MORTON, ORDER_ROWS = 0, 1, 2
G_FP32, G_FP64, GATHER_TABLE, GATHER_TABLE_FREE, GATHER_PASS = 0x1, 0x2, 0x4, 0x8, 0x10

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsem.so")


class SemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sem error {code}: {msg}")
        self.code = code


class CgOpts(C.Structure):
    _fields_ = [("prec", C.c_int), ("geom", C.c_int), ("tol", C.c_double),
                ("max_iter", C.c_int), ("fixed_iters", C.c_int), ("inner_tol", C.c_double),
                ("max_outer", C.c_int), ("poll_every", C.c_int), ("use_graph", C.c_int),
                ("true_residual", C.c_int), ("hist_rho", C.c_void_p),
                ("hist_alpha", C.c_void_p), ("hist_len", C.c_int),
                ("kernel_ms", C.c_void_p), ("precond", C.c_int)]


class CgResult(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer", C.c_int), ("converged", C.c_int),
                ("status", C.c_int), ("rel_res_recursive", C.c_double),
                ("rel_res_true", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MeshInfo(C.Structure):
    _fields_ = [("n_elem", C.c_int64), ("order_N", C.c_int32), ("n_local", C.c_int64),
                ("n_glob", C.c_int64), ("n_shared", C.c_int64), ("n_groups", C.c_int64),
                ("n_dirichlet", C.c_int64), ("device_bytes", C.c_size_t),
                ("gs_in_update", C.c_int32), ("gs_table_free", C.c_int32)]


_lib = None
EXPORTS = ["sem_mesh_create", "sem_mesh_destroy", "sem_mesh_info", "sem_ax", "sem_gs",
           "sem_dot", "sem_dot_noalloc", "sem_diag", "sem_element_order", "sem_coords", "sem_rhs", "sem_cg_solve", "sem_batch_create",
           "sem_batch_destroy", "sem_batch_solve", "sem_server_create", "sem_server_destroy",
           "sem_server_add", "sem_server_step", "sem_mesh_footprint", "sem_ax_shape_set",
           "sem_ax_shape_get", "sem_ax_engine_set", "sem_ax_engine_get", "sem_set_cache_bytes",
           "sem_last_error", "sem_version"]


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libsem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: run paper_2108_12188_amd/build.py "
                           "(or __graft_entry__.build()) first")
    L = C.CDLL(_LIB_PATH)
    vp, i64, i32, u32 = C.c_void_p, C.c_int64, C.c_int, C.c_uint32
    L.sem_mesh_create.argtypes = [i64, i32, vp, vp, vp, u32, vp, C.POINTER(vp)]
    L.sem_mesh_destroy.argtypes = [vp]
    L.sem_mesh_destroy.restype = None
    L.sem_element_order.argtypes = [i64, vp, i32, vp]
    L.sem_mesh_info.argtypes = [vp, C.POINTER(MeshInfo)]
    L.sem_ax.argtypes = [vp, i32, i32, vp, vp, vp]
    L.sem_gs.argtypes = [vp, i32, vp, i32, vp]
    L.sem_dot.argtypes = [vp, i32, vp, vp, vp, vp]
    L.sem_dot_noalloc.argtypes = [vp, i32, vp, vp, vp, vp]
    L.sem_coords.argtypes = [vp, vp, vp]
    L.sem_diag.argtypes = [vp, vp, vp]
    L.sem_rhs.argtypes = [vp, i32, vp, vp, vp]
    L.sem_cg_solve.argtypes = [vp, C.POINTER(CgOpts), vp, vp, C.POINTER(CgResult), vp]
    L.sem_batch_create.argtypes = [i32, vp, C.POINTER(vp)]
    L.sem_batch_destroy.argtypes = [vp]
    L.sem_batch_destroy.restype = None
    L.sem_batch_solve.argtypes = [vp, C.POINTER(CgOpts), vp, vp, vp, vp]
    L.sem_server_create.argtypes = [C.POINTER(CgOpts), i32, C.POINTER(vp)]
    L.sem_server_destroy.argtypes = [vp]
    L.sem_server_destroy.restype = None
    L.sem_server_add.argtypes = [vp, vp, vp, vp, i64, vp]
    L.sem_server_step.argtypes = [vp, vp, vp, i32, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.sem_mesh_footprint.argtypes = [i64, i32, u32, i32, C.POINTER(C.c_size_t)]
    L.sem_ax_shape_set.argtypes = [i32, i32, i32, i32]
    L.sem_ax_shape_get.argtypes = [i32, i32, i32, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                   C.POINTER(C.c_size_t)]
    L.sem_ax_engine_set.argtypes = [i32, i32, i32, i32]
    L.sem_ax_engine_get.argtypes = [i32, i32, i32, C.POINTER(C.c_int)]
    L.sem_set_cache_bytes.argtypes = [C.c_int64]
    L.sem_last_error.restype = C.c_char_p
    L.sem_last_error.argtypes = []
    L.sem_version.restype = C.c_char_p
    L.sem_version.argtypes = []
    for name in ("sem_mesh_create", "sem_mesh_info", "sem_ax", "sem_gs", "sem_dot", "sem_dot_noalloc",
                 "sem_coords", "sem_rhs", "sem_cg_solve", "sem_batch_create", "sem_batch_solve",
                 "sem_server_create", "sem_server_add", "sem_server_step", "sem_mesh_footprint",
                 "sem_ax_shape_set", "sem_ax_shape_get", "sem_ax_engine_set",
                 "sem_ax_engine_get", "sem_diag", "sem_element_order", "sem_set_cache_bytes"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def version() -> str:
    return lib().sem_version().decode()


def _check(code: int):
    if code != 0:
        raise SemError(code, lib().sem_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the SEM library needs a HIP device (torch.cuda.is_available() is False)")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _prec_of(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return FP32
    if t.dtype == torch.float64:
        return FP64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev_vec(t, n, name):
    if not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous device tensor of {n} entries")
    return C.c_void_p(t.data_ptr())


class Mesh:
    """A mesh on the current HIP device (owns all device-side mesh data).

    sem_mesh_create: g_fp32 / g_fp64 keep precomputed geometric factors in
    that precision; gather_table / table_free choose the form of the
    gather-scatter inside CG (per-point table, or position-derived at odd
    N) instead of the size rule (same results either way); gather_pass runs
    it as a pass of its own, the paper's schedule."""

    def __init__(self, vert, glob_id, dirichlet, N: int, g_fp32: bool = True,
                 g_fp64: bool = False, stream=None, gather_table: bool = False,
                 table_free: bool = False, gather_pass: bool = False):
        _torch()
        vert = np.ascontiguousarray(vert, dtype=np.float64)
        gid = np.ascontiguousarray(glob_id, dtype=np.int64)
        dr = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
        E = vert.shape[0]
        if vert.shape != (E, 8, 3) or gid.size != E * (N + 1) ** 3:
            raise ValueError("vert must be [E][8][3] and glob_id [E][(N+1)^3]")
        flags = ((G_FP32 if g_fp32 else 0) | (G_FP64 if g_fp64 else 0) |
                 (GATHER_TABLE if gather_table else 0) | (GATHER_TABLE_FREE if table_free else 0) |
                 (GATHER_PASS if gather_pass else 0))
        h = C.c_void_p()
        _check(lib().sem_mesh_create(E, N, vert.ctypes.data, gid.ctypes.data,
                                     None if dr is None else dr.ctypes.data, flags,
                                     _stream(stream), C.byref(h)))
        self._h = h
        self.N = N
        self.E = E
        self.n = E * (N + 1) ** 3

    @classmethod
    def from_box(cls, box, **kw):
        return cls(box.vert, box.glob_id, box.dirichlet, box.N, **kw)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("mesh was closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().sem_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = MeshInfo()
        _check(lib().sem_mesh_info(self.handle, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in MeshInfo._fields_}

    # -- operator pieces ---------------------------------------------------
    def ax(self, u, w=None, geom: int = PRECOMPUTED, stream=None):
        torch = _torch()
        if w is None:
            w = torch.empty_like(u)
        _check(lib().sem_ax(self.handle, _prec_of(u), geom, _dev_vec(u, self.n, "u"),
                            _dev_vec(w, self.n, "w"), _stream(stream)))
        return w

    def gs(self, w, mask: bool = True, stream=None):
        _check(lib().sem_gs(self.handle, _prec_of(w), _dev_vec(w, self.n, "w"),
                            1 if mask else 0, _stream(stream)))
        return w

    def dot(self, a, b, out=None, stream=None):
        torch = _torch()
        o = out if out is not None else torch.empty(1, dtype=torch.float64, device=a.device)
        _check(lib().sem_dot(self.handle, _prec_of(a), _dev_vec(a, self.n, "a"),
                             _dev_vec(b, self.n, "b"), C.c_void_p(o.data_ptr()),
                             _stream(stream)))
        return o if out is not None else float(o.item())

    def dot_noalloc(self, a, b, out, stream=None):
        """<a, b, c> into the one-element float64 device tensor `out`
        without any device allocation by the library (sem_dot_noalloc)."""
        _check(lib().sem_dot_noalloc(self.handle, _prec_of(a), _dev_vec(a, self.n, "a"),
                                     _dev_vec(b, self.n, "b"), _dev_vec(out, 1, "out"),
                                     _stream(stream)))
        return out

    def diag(self, stream=None):
        """Diagonal of the assembled operator in local form (float64 device
        tensor; the Jacobi preconditioner's M)."""
        torch = _torch()
        d = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(lib().sem_diag(self.handle, C.c_void_p(d.data_ptr()), _stream(stream)))
        return d

    def coords(self, stream=None):
        torch = _torch()
        xyz = torch.empty(3 * self.n, dtype=torch.float64, device="cuda")
        _check(lib().sem_coords(self.handle, C.c_void_p(xyz.data_ptr()), _stream(stream)))
        return xyz.view(3, self.n)

    def rhs(self, f, prec: int = FP64, stream=None):
        """b = mask(QQ^T (B f)) for a source f (float64 device tensor)."""
        torch = _torch()
        dt = torch.float32 if prec == FP32 else torch.float64
        b = torch.empty(self.n, dtype=dt, device=f.device)
        _check(lib().sem_rhs(self.handle, prec, _dev_vec(f, self.n, "f"),
                             C.c_void_p(b.data_ptr()), _stream(stream)))
        return b

    def cg_solve(self, b, x=None, prec: int | None = None, geom: int = PRECOMPUTED,
                 tol: float = 1e-8, max_iter: int = 100000, fixed_iters: int = 0,
                 inner_tol: float = 0.0, max_outer: int = 0, poll_every: int = 0,
                 use_graph: bool = True, true_residual: bool = False, history: int = 0,
                 kernel_times: bool = False, precond: int = PRECOND_NONE, stream=None):
        """Algorithm 1 (or its mixed-precision refinement), optionally
        Jacobi-preconditioned.  Returns (x, result dict)."""
        torch = _torch()
        if prec is None:
            prec = _prec_of(b)
        want = torch.float32 if prec == FP32 else torch.float64
        if b.dtype != want:
            raise TypeError("b has the wrong dtype for the requested precision")
        if x is None:
            x = torch.zeros_like(b)
        opts = CgOpts(prec=prec, geom=geom, tol=tol, max_iter=max_iter,
                      fixed_iters=fixed_iters, inner_tol=inner_tol, max_outer=max_outer,
                      poll_every=poll_every, use_graph=1 if use_graph else 0,
                      true_residual=1 if true_residual else 0, hist_len=0, precond=precond)
        hr = ha = None
        if history > 0:
            hr = np.zeros(history)
            ha = np.zeros(history)
            opts.hist_rho = hr.ctypes.data
            opts.hist_alpha = ha.ctypes.data
            opts.hist_len = history
        km = None
        if kernel_times:
            km = np.zeros(3)
            opts.kernel_ms = km.ctypes.data
        res = CgResult()
        code = lib().sem_cg_solve(self.handle, C.byref(opts), _dev_vec(b, self.n, "b"),
                                  _dev_vec(x, self.n, "x"), C.byref(res), _stream(stream))
        out = res.as_dict()
        if km is not None:
            out["kernel_ms"] = {"ax": km[0], "gs": km[1], "update": km[2]}
        if history > 0:
            k = min(history, res.iters + 1)
            out["hist_rho"] = hr[:k].copy()
            out["hist_alpha"] = ha[:k].copy()
        if code == -5:
            out["breakdown"] = True
            return x, out
        _check(code)
        return x, out


class Batch:
    """Independent meshes solved together (one batched launch per kernel type
    and CG iteration).  Each problem's result is bitwise that of its own
    Mesh.cg_solve with the same options."""

    def __init__(self, meshes):
        self.meshes = list(meshes)
        arr = (C.c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        h = C.c_void_p()
        _check(lib().sem_batch_create(len(self.meshes), arr, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().sem_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, bs, xs=None, prec: int = MIXED, geom: int = PRECOMPUTED, tol: float = 1e-8,
              max_iter: int = 100000, fixed_iters: int = 0, inner_tol: float = 0.0,
              max_outer: int = 0, poll_every: int = 0, use_graph: bool = True, stream=None):
        """Returns (xs, list of result dicts)."""
        torch = _torch()
        P = len(self.meshes)
        if len(bs) != P:
            raise ValueError("one right-hand side per mesh")
        want = torch.float32 if prec == FP32 else torch.float64
        if xs is None:
            xs = [torch.zeros_like(b) for b in bs]
        for m, b, x in zip(self.meshes, bs, xs):
            if b.dtype != want or x.dtype != want:
                raise TypeError("b and x must match the precision")
            _dev_vec(b, m.n, "b")
            _dev_vec(x, m.n, "x")
        barr = (C.c_void_p * P)(*[b.data_ptr() for b in bs])
        xarr = (C.c_void_p * P)(*[x.data_ptr() for x in xs])
        res = (CgResult * P)()
        opts = CgOpts(prec=prec, geom=geom, tol=tol, max_iter=max_iter, fixed_iters=fixed_iters,
                      inner_tol=inner_tol, max_outer=max_outer, poll_every=poll_every,
                      use_graph=1 if use_graph else 0, true_residual=0, hist_len=0)
        code = lib().sem_batch_solve(self._h, C.byref(opts), barr, xarr, res, _stream(stream))
        out = [r.as_dict() for r in res]
        if code == -5:
            return xs, out
        _check(code)
        return xs, out


def ax_shape_set(N: int, prec: int, geom: int, elems_per_block: int):
    """Tile shape (elements per workgroup) of the local operator; 0 = default."""
    _check(lib().sem_ax_shape_set(N, prec, geom, elems_per_block))


def ax_shape_get(N: int, prec: int, geom: int) -> dict:
    e, t, l = C.c_int(), C.c_int(), C.c_size_t()
    _check(lib().sem_ax_shape_get(N, prec, geom, C.byref(e), C.byref(t), C.byref(l)))
    return {"elems_per_block": e.value, "threads": t.value, "lds_bytes": int(l.value)}


ENGINE_DEFAULT, ENGINE_VALU, ENGINE_MFMA = 0, 1, 2


def ax_engine_set(N: int, prec: int, geom: int, engine: int):
    """Contraction engine of the local operator (VALU FMA or matrix cores)."""
    _check(lib().sem_ax_engine_set(N, prec, geom, engine))


def set_cache_bytes(nbytes: int = 0):
    """Cache size the CG drivers assume when they choose non-temporal p and x
    accesses (sem_set_cache_bytes; 0 = 256 MiB, the Infinity Cache)."""
    _check(lib().sem_set_cache_bytes(int(nbytes)))


def ax_engine_get(N: int, prec: int, geom: int) -> int:
    e = C.c_int()
    _check(lib().sem_ax_engine_get(N, prec, geom, C.byref(e)))
    return e.value


def element_order(vert, kind: int = ORDER_HILBERT) -> np.ndarray:
    """Element permutation by the element centroids, along a space-filling
    curve (ORDER_HILBERT, ORDER_MORTON) or in rows (ORDER_ROWS)
    (sem_element_order; host only): perm[k] is the input element placed at
    position k."""
    v = np.ascontiguousarray(vert, dtype=np.float64)
    if v.ndim != 3 or v.shape[1:] != (8, 3):
        raise ValueError("vert must be [E][8][3]")
    perm = np.empty(v.shape[0], dtype=np.int64)
    _check(lib().sem_element_order(v.shape[0], C.c_void_p(v.ctypes.data), kind,
                                   C.c_void_p(perm.ctypes.data)))
    return perm


def permute_elements(perm, *arrays):
    """The element-major arrays in the order perm: arrays whose first axis is
    the element (vertices [E][8][3], scatter map and Dirichlet flags
    [E][P^3]) are indexed along it; flat local vectors [E * P^3] by element
    blocks."""
    E = len(perm)
    out = []
    for a in arrays:
        a = np.asarray(a)
        if a.ndim >= 2 and a.shape[0] == E:
            out.append(np.ascontiguousarray(a[perm]))
        else:
            out.append(np.ascontiguousarray(a.reshape(E, -1)[perm].ravel()))
    return out


def mesh_footprint(n_elem: int, N: int, g_fp32: bool = True, g_fp64: bool = False,
                   prec: int = MIXED) -> int:
    """Upper bound of the device bytes of a mesh plus the work vectors of a solve."""
    out = C.c_size_t()
    flags = (G_FP32 if g_fp32 else 0) | (G_FP64 if g_fp64 else 0)
    _check(lib().sem_mesh_footprint(n_elem, N, flags, prec, C.byref(out)))
    return int(out.value)


class Server:
    """Continuous-batching mixed-precision solver (see sem_server_* in sem.h)."""

    def __init__(self, tol: float = 1e-8, geom: int = PRECOMPUTED, inner_tol: float = 0.0,
                 max_outer: int = 0, max_iter: int = 0, round_iters: int = 16):
        _torch()
        opts = CgOpts(prec=MIXED, geom=geom, tol=tol, max_iter=max_iter, fixed_iters=0,
                      inner_tol=inner_tol, max_outer=max_outer, poll_every=0, use_graph=0,
                      true_residual=0, hist_len=0)
        h = C.c_void_p()
        _check(lib().sem_server_create(C.byref(opts), round_iters, C.byref(h)))
        self._h = h
        self._held = {}

    def add(self, mesh: "Mesh", b, x, tag: int, stream=None):
        """Queue a request; the server reads b and x after the work already
        enqueued on `stream` (default: the current stream) has finished."""
        _dev_vec(b, mesh.n, "b")
        _dev_vec(x, mesh.n, "x")
        _check(lib().sem_server_add(self._h, mesh.handle, C.c_void_p(b.data_ptr()),
                                    C.c_void_p(x.data_ptr()), tag, _stream(stream)))
        self._held[tag] = (mesh, b, x)

    def step(self, cap: int = 256):
        """One round; returns (list of (tag, result dict), requests still held)."""
        tags = (C.c_int64 * cap)()
        res = (CgResult * cap)()
        nd = C.c_int()
        na = C.c_int()
        _check(lib().sem_server_step(self._h, tags, res, cap, C.byref(nd), C.byref(na)))
        done = []
        for q in range(nd.value):
            t = int(tags[q])
            self._held.pop(t, None)
            done.append((t, res[q].as_dict()))
        return done, na.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().sem_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
