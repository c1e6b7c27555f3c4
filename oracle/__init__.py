"""FP64 CPU oracle of the SEM Poisson CG hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library (``paper_2108_12188_amd``) and never imports it.

The arithmetic lives in ``sem_oracle.c`` (plain C, FP64); this module only
marshals NumPy arrays into it and bundles the per-mesh quantities.
Readings of the paper taken here are listed at the top of ``sem_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sem_oracle.c")
_LIB = os.path.join(_HERE, "libsem_oracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_bp = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction into FMA)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]
        L.or_set_num_threads.restype = None
        L.or_gll.argtypes = [C.c_int, _dp, _dp]
        L.or_gll.restype = C.c_int
        L.or_deriv.argtypes = [C.c_int, _dp, _dp]
        L.or_deriv.restype = C.c_int
        L.or_geom.argtypes = [C.c_long, C.c_int, _dp, _dp, _dp, _dp, C.c_void_p]
        L.or_geom.restype = C.c_long
        L.or_coords.argtypes = [C.c_long, C.c_int, _dp, _dp, _dp]
        L.or_ax_local.argtypes = [C.c_long, C.c_int, _dp, _dp, _dp, _dp]
        L.or_gs.argtypes = [C.c_long, _ip, C.c_long, _dp, _dp]
        L.or_mask.argtypes = [C.c_long, _bp, _dp]
        L.or_multiplicity.argtypes = [C.c_long, _ip, C.c_long, _dp]
        L.or_dot.argtypes = [C.c_long, _dp, _dp, _dp]
        L.or_dot.restype = C.c_double
        L.or_apply_A.argtypes = [C.c_long, C.c_int, _dp, _dp, _ip, C.c_long, _bp, _dp, _dp]
        L.or_cg.argtypes = [C.c_long, C.c_int, _dp, _dp, _ip, C.c_long, _bp, _dp, _dp, _dp,
                            C.c_double, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_cg.restype = C.c_int
        L.or_diag_A.argtypes = [C.c_long, C.c_int, _dp, _dp, _ip, C.c_long, _dp]
        L.or_pcg.argtypes = [C.c_long, C.c_int, _dp, _dp, _ip, C.c_long, _bp, _dp, _dp, _dp,
                             _dp, C.c_double, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                             C.c_void_p]
        L.or_pcg.restype = C.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(k: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (for timing)."""
    lib().or_set_num_threads(int(k))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def gll(N: int):
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    if lib().or_gll(N, xi, w) != 0:
        raise ValueError(f"unsupported order N={N}")
    return xi, w


def deriv(N: int, xi=None):
    if xi is None:
        xi, _ = gll(N)
    D = np.zeros((N + 1) * (N + 1))
    if lib().or_deriv(N, _f64(xi), D) != 0:
        raise ValueError(f"unsupported order N={N}")
    return D.reshape(N + 1, N + 1)


def geom(vert, N: int, xi=None, w=None):
    """G [E][6][P^3] and B [E][P^3]; raises on a non-positive Jacobian."""
    if xi is None:
        xi, w = gll(N)
    vert = _f64(vert)
    E = vert.shape[0]
    P3 = (N + 1) ** 3
    G = np.zeros((E, 6, P3))
    B = np.zeros((E, P3))
    bad = lib().or_geom(E, N, vert, _f64(xi), _f64(w), G, B.ctypes.data)
    if bad >= 0:
        raise ValueError(f"non-positive Jacobian in element {bad}")
    return G, B


def coords(vert, N: int, xi=None):
    if xi is None:
        xi, _ = gll(N)
    vert = _f64(vert)
    E = vert.shape[0]
    xyz = np.zeros((3, E * (N + 1) ** 3))
    lib().or_coords(E, N, vert, _f64(xi), xyz)
    return xyz


def ax_local(N: int, D, G, u):
    G = _f64(G)
    E = G.shape[0]
    w = np.zeros(E * (N + 1) ** 3)
    lib().or_ax_local(E, N, _f64(D), G, _f64(u).ravel(), w)
    return w


def gs(glob_id, n_glob: int, w):
    w = _f64(w).ravel().copy()
    gid = np.ascontiguousarray(glob_id, dtype=np.int64).ravel()
    lib().or_gs(w.size, gid, n_glob, w, np.zeros(n_glob))
    return w


def mask(dirichlet, w):
    w = _f64(w).ravel().copy()
    lib().or_mask(w.size, np.ascontiguousarray(dirichlet, dtype=np.uint8).ravel(), w)
    return w


def multiplicity(glob_id, n_glob: int):
    gid = np.ascontiguousarray(glob_id, dtype=np.int64).ravel()
    m = np.zeros(gid.size)
    lib().or_multiplicity(gid.size, gid, n_glob, m)
    return m


def dot(a, b, m):
    a, b, m = _f64(a).ravel(), _f64(b).ravel(), _f64(m).ravel()
    return lib().or_dot(a.size, a, b, m)


class Problem:
    """One mesh with every per-mesh quantity the oracle needs (FP64)."""

    def __init__(self, mesh):
        self.mesh = mesh
        self.N = mesh.N
        self.E = mesh.E
        self.n = mesh.n_local
        self.n_glob = mesh.n_glob
        self.xi, self.w = gll(self.N)
        self.D = deriv(self.N, self.xi)
        self.G, self.B = geom(mesh.vert, self.N, self.xi, self.w)
        self.glob_id = np.ascontiguousarray(mesh.glob_id.ravel(), dtype=np.int64)
        self.dirichlet = np.ascontiguousarray(mesh.dirichlet.ravel(), dtype=np.uint8)
        self.m = multiplicity(self.glob_id, self.n_glob)

    # operator pieces -------------------------------------------------
    def ax_local(self, u):
        return ax_local(self.N, self.D, self.G, u)

    def gs(self, w):
        return gs(self.glob_id, self.n_glob, w)

    def mask(self, w):
        return mask(self.dirichlet, w)

    def apply_A(self, u):
        w = np.zeros(self.n)
        lib().or_apply_A(self.E, self.N, _f64(self.D), self.G, self.glob_id, self.n_glob,
                         self.dirichlet, _f64(u).ravel(), w)
        return w

    def dot(self, a, b):
        return dot(a, b, self.m)

    # right-hand sides ------------------------------------------------
    def coords(self):
        return coords(self.mesh.vert, self.N, self.xi)

    def rhs_manufactured(self):
        """b = mask(QQ^T (B f)) for f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z),
        the forcing of -Laplace(u) = f with u = sin sin sin; returns (b, u_exact)."""
        x, y, z = self.coords()
        u = np.sin(math.pi * x) * np.sin(math.pi * y) * np.sin(math.pi * z)
        f = 3.0 * math.pi ** 2 * u
        b = self.mask(self.gs(self.B.ravel() * f))
        return b, u

    # solver ------------------------------------------------------------
    def cg(self, b, x0=None, tol=1e-8, max_iter=10000, fixed=0, history=True):
        """Algorithm 1; returns (x, iters, hist) with hist = dict(rho, alpha, beta)."""
        x = np.zeros(self.n) if x0 is None else self.mask(x0)
        b = _f64(b).ravel()
        L = (fixed if fixed > 0 else max_iter) + 1
        rho = np.zeros(L)
        alpha = np.zeros(L)
        beta = np.zeros(L)
        it = lib().or_cg(self.E, self.N, _f64(self.D), self.G, self.glob_id, self.n_glob,
                         self.dirichlet, self.m, b, x, tol, max_iter, fixed,
                         rho.ctypes.data if history else None,
                         alpha.ctypes.data if history else None,
                         beta.ctypes.data if history else None)
        hist = {"rho": rho[:it + 1], "alpha": alpha[:it + 1], "beta": beta[:it + 1]}
        return x, it, hist

    # Jacobi preconditioner (f4) --------------------------------------
    def diag_A(self):
        """Diagonal of the assembled operator Q^T A_L Q, in local form
        (unmasked)."""
        d = np.zeros(self.n)
        lib().or_diag_A(self.E, self.N, _f64(self.D), self.G, self.glob_id, self.n_glob, d)
        return d

    def jacobi_minv(self):
        """M^-1 of the Jacobi preconditioner: 1/diag on the free points, 0 on
        the Dirichlet points."""
        d = self.diag_A()
        return np.where(self.dirichlet.astype(bool), 0.0, 1.0 / d)

    def pcg(self, b, minv=None, x0=None, tol=1e-8, max_iter=10000, fixed=0):
        """Jacobi-preconditioned Algorithm 1; returns (x, iters, hist) with
        hist = dict(rho = <r,r,c>, alpha, beta)."""
        minv = self.jacobi_minv() if minv is None else _f64(minv).ravel()
        x = np.zeros(self.n) if x0 is None else self.mask(x0)
        b = _f64(b).ravel()
        L = (fixed if fixed > 0 else max_iter) + 1
        rho, alpha, beta = np.zeros(L), np.zeros(L), np.zeros(L)
        it = lib().or_pcg(self.E, self.N, _f64(self.D), self.G, self.glob_id, self.n_glob,
                          self.dirichlet, self.m, minv, b, x, tol, max_iter, fixed,
                          rho.ctypes.data, alpha.ctypes.data, beta.ctypes.data)
        return x, it, {"rho": rho[:it + 1], "alpha": alpha[:it + 1], "beta": beta[:it + 1]}

    def true_rel_residual(self, b, x):
        r = _f64(b).ravel() - self.apply_A(x)
        nb = self.dot(b, b)
        return math.sqrt(self.dot(r, r) / nb) if nb > 0 else math.sqrt(self.dot(r, r))
