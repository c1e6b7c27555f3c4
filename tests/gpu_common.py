"""Helpers shared by the GPU parity tests: the same seeded mesh goes to the
oracle (CPU, FP64) and to the HIP library through the C ABI."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    """Print and flush the case name before a GPU step."""
    print(*a, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    return torch


def to_dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_norm(got, ref):
    d = np.linalg.norm(got - ref)
    r = np.linalg.norm(ref)
    return d / r if r > 0 else d


def oracle_ax_elems(mesh, u, elems):
    """Oracle A_L of the listed elements only (geometry and operator computed
    element by element from the same vertices): [len(elems)][P^3]."""
    import oracle
    N = mesh.N
    P3 = (N + 1) ** 3
    xi, w = oracle.gll(N)
    D = oracle.deriv(N, xi)
    G, _ = oracle.geom(mesh.vert[elems], N, xi, w)
    U = np.ascontiguousarray(u.reshape(-1, P3)[elems])
    return oracle.ax_local(N, D, G, U.ravel()).reshape(len(elems), P3)
