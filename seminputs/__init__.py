"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the spectral-element method: no GLL
points, no derivative matrix, no geometric factors, no operator.  It only
produces what a mesh file and a right-hand-side file would hold for the
paper's workload (a cubic domain of linearly deformed hexahedra, Sec. 6 and
Sec. 5.1 of the paper):

* element vertex coordinates ``vert[E][8][3]`` (vertex ``a + 2b + 4c`` sits
  at reference corner ``(2a-1, 2b-1, 2c-1)``), rounded once to FP32 so both
  precisions see identical geometry;
* the scatter map ``glob_id[E][P^3]`` (local point ``i + P*(j + P*k)`` of an
  element -> global point), i.e. the operator Q of Eq. (5);
* the Dirichlet flags ``dirichlet[E][P^3]`` (1 on the boundary of the box);
* random continuous right-hand sides and the batch / arrival schedules of the
  batched and serving workloads.

Index manipulation (element permutation, rotation of an element's local
frame) is done here too, because an unstructured mesh generator would emit
such meshes.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "BoxMesh",
    "box_mesh",
    "graded_z",
    "random_global_rhs",
    "batch_problems",
    "arrival_times",
    "MESH_SEED_BASE",
    "RHS_SEED",
]

MESH_SEED_BASE = 2108
RHS_SEED = 12188


@dataclass
class BoxMesh:
    nx: int
    ny: int
    nz: int
    N: int
    vert: np.ndarray          # float64 [E][8][3], values exactly representable in FP32
    glob_id: np.ndarray       # int64 [E][P^3]
    dirichlet: np.ndarray     # uint8 [E][P^3]
    n_glob: int
    perturb: float = 0.0
    seed: int = 0
    info: dict = field(default_factory=dict)

    @property
    def E(self) -> int:
        return self.vert.shape[0]

    @property
    def P(self) -> int:
        return self.N + 1

    @property
    def n_local(self) -> int:
        return self.E * self.P ** 3


def _rotations():
    """The 24 proper rotations of the cube as (axis permutation, signs)."""
    out = []
    for perm in itertools.permutations(range(3)):
        # parity of the permutation
        inv = sum(1 for a in range(3) for b in range(a + 1, 3) if perm[a] > perm[b])
        psign = -1 if inv % 2 else 1
        for signs in itertools.product((1, -1), repeat=3):
            if psign * signs[0] * signs[1] * signs[2] == 1:
                out.append((perm, signs))
    return out


_ROT = _rotations()


def _reorient_index(P: int, perm, signs) -> np.ndarray:
    """old local index for every new local index i' + P*(j' + P*k').

    New reference coordinate axis ``perm[d]`` (possibly flipped) becomes old
    axis ``d``; index flips map GLL index t to P-1-t (the GLL set is
    symmetric), so the map stays on the node set.
    """
    idx = np.arange(P)
    kk, jj, ii = np.meshgrid(idx, idx, idx, indexing="ij")
    new = (ii.ravel(), jj.ravel(), kk.ravel())
    old = []
    for d in range(3):
        t = new[perm[d]]
        old.append(t if signs[d] > 0 else (P - 1 - t))
    return old[0] + P * (old[1] + P * old[2])


def box_mesh(nx: int, ny: int, nz: int, N: int, perturb: float = 0.0,
             seed: int = 0, permute: bool = False, reorient: bool = False) -> BoxMesh:
    """Hexahedral mesh of the unit cube with ``nx*ny*nz`` elements of order N.

    perturb: every coordinate of every interior grid vertex is shifted by
    U(-perturb*h, +perturb*h) with h the grid spacing along that axis
    (PCG64(seed)); boundary vertices stay on the faces of the cube, so the
    deformed elements stay linear (trilinear) hexahedra.
    permute: elements are stored in a seeded random order.
    reorient: each element's local frame is rotated by one of the 24 proper
    cube rotations (seeded), as an unstructured mesh would hold it.
    """
    if min(nx, ny, nz) < 1 or N < 1:
        raise ValueError("box_mesh needs nx, ny, nz >= 1 and N >= 1")
    P = N + 1
    rng = np.random.Generator(np.random.PCG64(seed))
    gx = np.linspace(0.0, 1.0, nx + 1)
    gy = np.linspace(0.0, 1.0, ny + 1)
    gz = np.linspace(0.0, 1.0, nz + 1)
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")        # [nz+1][ny+1][nx+1]
    grid = np.stack([X, Y, Z], axis=-1)                      # [..][3]
    if perturb:
        h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
        noise = rng.uniform(-1.0, 1.0, size=grid.shape) * (perturb * h)
        interior = np.zeros(grid.shape[:3], dtype=bool)
        interior[1:-1, 1:-1, 1:-1] = True
        # a vertex on a face of the cube may still slide inside that face,
        # but we keep every boundary vertex fixed to keep the box exact
        grid = grid + noise * interior[..., None]
    grid = grid.astype(np.float32).astype(np.float64)

    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    E = ex.size
    vert = np.empty((E, 8, 3), dtype=np.float64)
    for c in range(2):
        for b in range(2):
            for a in range(2):
                vert[:, a + 2 * b + 4 * c, :] = grid[ez + c, ey + b, ex + a, :]

    idx = np.arange(P)
    kk, jj, ii = np.meshgrid(idx, idx, idx, indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()          # local point l = i + P(j + Pk)
    GX, GY = nx * N + 1, ny * N + 1
    px = ex[:, None] * N + ii[None, :]
    py = ey[:, None] * N + jj[None, :]
    pz = ez[:, None] * N + kk[None, :]
    glob_id = (px + GX * (py + GY * pz)).astype(np.int64)
    dirichlet = ((px == 0) | (px == nx * N) | (py == 0) | (py == ny * N)
                 | (pz == 0) | (pz == nz * N)).astype(np.uint8)
    n_glob = GX * GY * (nz * N + 1)

    if reorient:
        choice = rng.integers(0, len(_ROT), size=E)
        corner_maps = [_reorient_index(2, *r) for r in _ROT]
        point_maps = [_reorient_index(P, *r) for r in _ROT]
        for r in range(len(_ROT)):
            sel = np.nonzero(choice == r)[0]
            if sel.size == 0:
                continue
            vert[sel] = vert[sel][:, corner_maps[r], :]
            glob_id[sel] = glob_id[sel][:, point_maps[r]]
            dirichlet[sel] = dirichlet[sel][:, point_maps[r]]
    if permute:
        order = rng.permutation(E)
        vert, glob_id, dirichlet = vert[order], glob_id[order], dirichlet[order]

    return BoxMesh(nx=nx, ny=ny, nz=nz, N=N, vert=np.ascontiguousarray(vert),
                   glob_id=np.ascontiguousarray(glob_id),
                   dirichlet=np.ascontiguousarray(dirichlet), n_glob=int(n_glob),
                   perturb=perturb, seed=seed,
                   info={"permute": permute, "reorient": reorient})


def graded_z(mesh: BoxMesh, s: float = 3.0) -> BoxMesh:
    """The same mesh with its vertices moved along z by the monotone map
    z -> (z + s z^3) / (1 + s), which keeps the faces z = 0 and z = 1: the
    elements next to z = 0 become about 1 + 3s times thinner than those next
    to z = 1 (a boundary-layer grading), so the diagonal of the operator
    varies strongly over the mesh.  Coordinates are rounded to FP32 again;
    copies of a vertex map to the same point, so the mesh stays conforming.
    """
    import dataclasses
    vert = mesh.vert.copy()
    z = vert[..., 2]
    vert[..., 2] = (z + s * z ** 3) / (1.0 + s)
    vert = vert.astype(np.float32).astype(np.float64)
    info = dict(mesh.info)
    info["graded_z"] = s
    return dataclasses.replace(mesh, vert=np.ascontiguousarray(vert), info=info)


def random_global_rhs(mesh: BoxMesh, seed: int = RHS_SEED) -> np.ndarray:
    """Continuous, masked random right-hand side in local form.

    One value U[-1, 1] per global point (PCG64(seed)), rounded once to FP32,
    copied to every local copy of that point and zeroed on the Dirichlet
    boundary.  Returned as float64 holding FP32-representable values.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    bg = rng.uniform(-1.0, 1.0, size=mesh.n_glob).astype(np.float32).astype(np.float64)
    b = bg[mesh.glob_id.ravel()]
    b[mesh.dirichlet.ravel() != 0] = 0.0
    return b


def random_local(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Independent U[lo, hi] per local point (discontinuous), FP32-representable."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=n).astype(np.float32).astype(np.float64)


def batch_problems(count: int = 64, seed: int = MESH_SEED_BASE + 4,
                   e_lo: int = 8 ** 3, e_hi: int = 20 ** 3, orders=(5, 7, 9)):
    """Problem list of the batched workload.

    Element counts log-uniform in [e_lo, e_hi]; the box is
    nx = ny = round(cbrt(E*)), nz = max(1, round(E*/nx^2)); N uniform from
    ``orders``; each problem gets its own mesh seed.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for p in range(count):
        est = math.exp(rng.uniform(math.log(e_lo), math.log(e_hi)))
        nxy = max(1, int(round(est ** (1.0 / 3.0))))
        nz = max(1, int(round(est / (nxy * nxy))))
        N = int(orders[int(rng.integers(0, len(orders)))])
        out.append({"nx": nxy, "ny": nxy, "nz": nz, "N": N,
                    "seed": int(seed * 1000 + p), "rhs_seed": int(RHS_SEED + p)})
    return out


def arrival_times(count: int, rate: float, seed: int) -> np.ndarray:
    """Poisson-process arrival times (seconds) with the given rate (1/s)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=count)
    return np.cumsum(gaps)
