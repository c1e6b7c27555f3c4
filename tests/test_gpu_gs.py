"""Parity of the HIP gather-scatter, mask, weighted dot, coordinates and
right-hand side with the FP64 oracle (Sec. 3.1, Sec. 4.3, Algorithm 1).

FP64 gather-scatter sums every group in ascending local index, as the
oracle does, so the FP64 results are bitwise equal.  FP32 sums stay within
m * eps32 of the exact sum, componentwise.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_common import rel_norm, say, to_dev, to_host
from seminputs import box_mesh, random_global_rhs, random_local

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,shape", [(1, (3, 2, 2)), (3, (4, 3, 5)), (5, (3, 3, 3)),
                                     (7, (4, 4, 4)), (9, (2, 3, 2))])
def test_gs_fp64_bitwise(N, shape):
    import torch
    import paper_2108_12188_amd as sem
    say(f"gs fp64 N={N} shape={shape}")
    mesh = box_mesh(*shape, N, perturb=0.1, seed=7, permute=True, reorient=True)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh)
    v = random_local(mesh.n_local, seed=3)
    for mask in (False, True):
        ref = pr.gs(v)
        if mask:
            ref = pr.mask(ref)
        w = to_dev(v, torch.float64)
        gm.gs(w, mask=mask)
        assert np.array_equal(to_host(w), ref)
    inf = gm.info()
    assert inf["n_local"] == mesh.n_local
    assert inf["n_glob"] == len(np.unique(mesh.glob_id))
    assert inf["n_shared"] == int(np.sum(pr.m > 1))
    assert inf["n_dirichlet"] == int(mesh.dirichlet.sum())
    gm.close()


@pytest.mark.parametrize("N", [2, 7])
def test_gs_fp32(N):
    import torch
    import paper_2108_12188_amd as sem
    mesh = box_mesh(4, 3, 3, N, perturb=0.1, seed=8, permute=True)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh)
    v = random_local(mesh.n_local, seed=4).astype(np.float32)
    ref = pr.mask(pr.gs(v.astype(np.float64)))
    w = to_dev(v, torch.float32)
    gm.gs(w, mask=True)
    got = to_host(w)
    # |fl(sum) - sum| <= (m-1) eps32 sum |v_i| <= 8 eps32 m max|v|
    bound = 8 * 2.0 ** -24 * pr.m * np.max(np.abs(v))
    assert np.all(np.abs(got - ref) <= bound)
    gm.close()


def test_gs_single_element_has_no_groups():
    import torch
    import paper_2108_12188_amd as sem
    mesh = box_mesh(1, 1, 1, 4)
    gm = sem.Mesh.from_box(mesh)
    assert gm.info()["n_groups"] == 0
    v = random_local(mesh.n_local, seed=1)
    w = to_dev(v, torch.float64)
    gm.gs(w, mask=False)
    assert np.array_equal(to_host(w), v)
    gm.close()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_dot(dt):
    import torch
    import paper_2108_12188_amd as sem
    mesh = box_mesh(5, 4, 3, 6, perturb=0.1, seed=2)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh)
    a = random_local(mesh.n_local, seed=1)
    b = random_local(mesh.n_local, seed=2)
    tdt = torch.float64 if dt == "f64" else torch.float32
    if dt == "f32":
        a, b = a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
    got = gm.dot(to_dev(a, tdt), to_dev(b, tdt))
    ref = pr.dot(a, b)
    assert abs(got - ref) <= 1e-12 * np.sum(np.abs(a * b / pr.m))
    # bitwise reproducible
    assert gm.dot(to_dev(a, tdt), to_dev(b, tdt)) == got
    gm.close()


def test_coords_and_rhs():
    import torch
    import paper_2108_12188_amd as sem
    mesh = box_mesh(3, 4, 2, 5, perturb=0.1, seed=12, reorient=True)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh)
    xyz = to_host(gm.coords())
    ref = pr.coords()
    assert np.max(np.abs(xyz.reshape(3, -1) - ref)) < 1e-14
    x, y, z = (torch.as_tensor(ref[d], device="cuda") for d in range(3))
    f = 3 * math.pi ** 2 * torch.sin(math.pi * x) * torch.sin(math.pi * y) * torch.sin(math.pi * z)
    b64 = to_host(gm.rhs(f.contiguous(), prec=sem.FP64))
    bref, _ = pr.rhs_manufactured()
    assert rel_norm(b64, bref) < 1e-14
    b32 = to_host(gm.rhs(f.contiguous(), prec=sem.FP32))
    assert np.array_equal(b32, b64.astype(np.float32).astype(np.float64))
    gm.close()


def test_mesh_errors():
    import paper_2108_12188_amd as sem
    mesh = box_mesh(2, 1, 1, 3)
    vert = mesh.vert.copy()
    vert[1, [0, 1]] = vert[1, [1, 0]]
    with pytest.raises(sem.SemError) as ei:
        sem.Mesh(vert, mesh.glob_id, mesh.dirichlet, 3)
    assert ei.value.code == -4 and "element 1" in str(ei.value)
    d = mesh.dirichlet.copy()
    # make one copy of a shared boundary point disagree
    g = mesh.glob_id.ravel()
    shared = np.nonzero(np.bincount(g)[g] > 1)[0]
    dd = d.ravel()
    dd[shared[0]] ^= 1
    with pytest.raises(sem.SemError) as ei:
        sem.Mesh(mesh.vert, mesh.glob_id, dd.reshape(d.shape), 3)
    assert ei.value.code == -1
    with pytest.raises(ValueError):
        sem.Mesh(mesh.vert, mesh.glob_id, mesh.dirichlet, 4)
    # an empty mesh passes the shape check and is refused by the library
    with pytest.raises(sem.SemError) as ei:
        sem.Mesh(np.zeros((0, 8, 3)), np.zeros((0, 64), np.int64), None, 3)
    assert ei.value.code == -1 and "n_elem" in str(ei.value)
    big = box_mesh(1, 1, 1, 12)
    with pytest.raises(sem.SemError) as ei:
        sem.Mesh.from_box(big)
    assert ei.value.code == -6
