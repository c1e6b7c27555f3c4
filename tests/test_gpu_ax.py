"""Parity of the HIP local operator (sem_ax) with the FP64 oracle.

Eq. 4-5: w_e = D^T G^e D u_e.  Precomputed and on-the-fly G, FP64 and
FP32, every built order, meshes that span several blocks and end in a
ragged block, deformed, permuted and rotated elements.  Bars: FP64 within
1e-12 normwise (different rounding order only); FP32 within 1e-5 normwise
(the stated FP32 bound of the operator).
"""
import numpy as np
import pytest

import oracle
from gpu_common import oracle_ax_elems, rel_norm, say, to_dev, to_host
from seminputs import box_mesh, random_local

pytestmark = pytest.mark.gpu


def _mesh(N, shape, seed=3):
    return box_mesh(*shape, N, perturb=0.1, seed=seed, permute=True, reorient=True)


def _smooth(pr):
    x, y, z = pr.coords()
    return np.sin(2.1 * x + 0.3) * np.cos(1.3 * y) * np.exp(0.4 * z)


# element counts chosen to span several blocks with a ragged last block
CASES = [(1, (5, 3, 4)), (2, (4, 3, 3)), (3, (5, 4, 2)), (4, (3, 3, 3)), (5, (4, 3, 2)),
         (6, (3, 3, 2)), (7, (4, 3, 3)), (8, (3, 3, 2)), (9, (3, 2, 2)), (10, (3, 2, 2)),
         (11, (2, 2, 2))]


@pytest.mark.parametrize("N,shape", CASES)
@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_ax_fp64(N, shape, geom):
    import torch
    import paper_2108_12188_amd as sem
    say(f"ax fp64 N={N} shape={shape} geom={geom}")
    mesh = _mesh(N, shape)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh, g_fp32=True, g_fp64=True)
    for u in (random_local(mesh.n_local, seed=N), _smooth(pr)):
        ref = pr.ax_local(u)
        w = gm.ax(to_dev(u, torch.float64), geom=geom)
        torch.cuda.synchronize()
        got = to_host(w)
        assert rel_norm(got, ref) < 1e-12
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    gm.close()


@pytest.mark.parametrize("N,shape", CASES)
@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_ax_fp32(N, shape, geom):
    import torch
    import paper_2108_12188_amd as sem
    say(f"ax fp32 N={N} shape={shape} geom={geom}")
    mesh = _mesh(N, shape, seed=5)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh)
    for u in (random_local(mesh.n_local, seed=10 + N), _smooth(pr)):
        u32 = u.astype(np.float32)
        ref = pr.ax_local(u32.astype(np.float64))
        w = gm.ax(to_dev(u32, torch.float32), geom=geom)
        torch.cuda.synchronize()
        assert rel_norm(to_host(w), ref) < 1e-5
    gm.close()


def test_ax_fp32_large_sampled():
    """32^3 elements, N = 7, +-10% deformed: the full-size operator, checked
    on 64 sampled elements that the oracle computes one by one."""
    import torch
    import paper_2108_12188_amd as sem
    say("ax fp32 32^3 N=7 sampled")
    mesh = box_mesh(32, 32, 32, 7, perturb=0.1, seed=2110)
    gm = sem.Mesh.from_box(mesh)
    u = random_local(mesh.n_local, seed=77).astype(np.float32)
    ud = to_dev(u, torch.float32)
    rng = np.random.default_rng(0)
    elems = np.sort(rng.choice(mesh.E, 64, replace=False))
    elems[-1] = mesh.E - 1
    ref = oracle_ax_elems(mesh, u.astype(np.float64), elems)
    for geom in (0, 1):
        w = to_host(gm.ax(ud, geom=geom)).reshape(mesh.E, -1)[elems]
        assert rel_norm(w, ref) < 1e-5, geom
    gm.close()


def test_ax_precomputed_and_otf_agree_fp64():
    import torch
    import paper_2108_12188_amd as sem
    mesh = _mesh(7, (3, 3, 3), seed=9)
    gm = sem.Mesh.from_box(mesh, g_fp32=False, g_fp64=True)
    u = to_dev(random_local(mesh.n_local, seed=1), torch.float64)
    a = to_host(gm.ax(u, geom=0))
    b = to_host(gm.ax(u, geom=1))
    assert rel_norm(a, b) < 1e-13
    gm.close()


def test_ax_missing_g_is_unsupported():
    import torch
    import paper_2108_12188_amd as sem
    mesh = box_mesh(2, 2, 2, 3)
    gm = sem.Mesh.from_box(mesh, g_fp32=False, g_fp64=False)
    u = torch.zeros(mesh.n_local, dtype=torch.float32, device="cuda")
    with pytest.raises(sem.SemError) as ei:
        gm.ax(u, geom=0)
    assert ei.value.code == -6
    gm.ax(u, geom=1)          # the on-the-fly form needs no stored G
    torch.cuda.synchronize()
    gm.close()
