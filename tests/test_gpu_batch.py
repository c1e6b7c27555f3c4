"""Batched solves: every problem of a batch (mixed element counts and
orders, one launch per kernel type per iteration) ends bitwise equal to its
own single-mesh solve, and meets its tolerance against the oracle."""
import math

import numpy as np
import pytest

import oracle
from gpu_common import rel_norm, say, to_dev, to_host
from seminputs import box_mesh, random_global_rhs

pytestmark = pytest.mark.gpu

SHAPES = [((3, 2, 2), 5), ((4, 3, 2), 7), ((2, 2, 2), 9), ((5, 4, 3), 3), ((2, 3, 2), 7)]


def _meshes(sem, g_fp32=True):
    boxes = [box_mesh(*sh, N, perturb=0.1, seed=40 + q, reorient=True, permute=True)
             for q, (sh, N) in enumerate(SHAPES)]
    return boxes, [sem.Mesh.from_box(b, g_fp32=g_fp32) for b in boxes]


def _manufactured(gm):
    import torch
    xyz = gm.coords()
    f = 3 * math.pi ** 2 * torch.sin(math.pi * xyz[0]) * torch.sin(math.pi * xyz[1]) \
        * torch.sin(math.pi * xyz[2])
    return f.contiguous()


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_batch_fp32_fixed_equals_solo(geom):
    import torch
    import paper_2108_12188_amd as sem
    say(f"batch fp32 fixed geom={geom}")
    boxes, gms = _meshes(sem)
    bs = [to_dev(random_global_rhs(b, seed=7 + q), torch.float32) for q, b in enumerate(boxes)]
    batch = sem.Batch(gms)
    xs, res = batch.solve(bs, prec=sem.FP32, geom=geom, fixed_iters=23)
    for q, gm in enumerate(gms):
        xq, rq = gm.cg_solve(bs[q], prec=sem.FP32, geom=geom, fixed_iters=23)
        assert res[q]["iters"] == 23 == rq["iters"]
        assert torch.equal(xs[q], xq), q
    batch.close()


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_batch_mixed_gather_forms_equal_solo(geom):
    """One batch holding meshes with the table-free gather (odd N, forced), with
    the per-point table (SEM_MESH_GATHER_TABLE, and an even order): every
    problem ends bitwise equal to its own solve, and the two forms of the
    same mesh to each other."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"batch mixed gather forms geom={geom}")
    b7 = box_mesh(3, 3, 2, 7, perturb=0.1, seed=60, reorient=True, permute=True)
    b4 = box_mesh(3, 2, 2, 4, perturb=0.1, seed=61, reorient=True, permute=True)
    b9 = box_mesh(2, 2, 3, 9, perturb=0.1, seed=62)
    gms = [sem.Mesh.from_box(b7, table_free=True), sem.Mesh.from_box(b7, gather_table=True),
           sem.Mesh.from_box(b4, table_free=True), sem.Mesh.from_box(b9, table_free=True)]
    assert [g.info()["gs_table_free"] for g in gms] == [1, 0, 0, 1]
    boxes = [b7, b7, b4, b9]
    bs = [to_dev(random_global_rhs(b, seed=70 + (q != 1) * q), torch.float32)
          for q, b in enumerate(boxes)]
    batch = sem.Batch(gms)
    xs, res = batch.solve(bs, prec=sem.FP32, geom=geom, fixed_iters=19)
    for q, gm in enumerate(gms):
        xq, rq = gm.cg_solve(bs[q], prec=sem.FP32, geom=geom, fixed_iters=19)
        assert res[q]["iters"] == 19 == rq["iters"]
        assert torch.equal(xs[q], xq), q
    assert torch.equal(xs[0], xs[1])
    batch.close()
    for g in gms:
        g.close()


def test_batch_fp32_tolerance_equals_solo_and_oracle():
    import torch
    import paper_2108_12188_amd as sem
    boxes, gms = _meshes(sem)
    bh = [random_global_rhs(b, seed=3 + q).astype(np.float32).astype(np.float64)
          for q, b in enumerate(boxes)]
    bs = [to_dev(v, torch.float32) for v in bh]
    batch = sem.Batch(gms)
    xs, res = batch.solve(bs, prec=sem.FP32, tol=1e-5, max_iter=5000)
    # the problems stop at different iterations, so stopped ones leave the
    # launches during the solve; a second solve on the same batch (its full
    # member list restored) gives the same results
    assert len({r["iters"] for r in res}) > 1
    xs2, res2 = batch.solve(bs, prec=sem.FP32, tol=1e-5, max_iter=5000)
    for q, gm in enumerate(gms):
        xq, rq = gm.cg_solve(bs[q], prec=sem.FP32, tol=1e-5, max_iter=5000)
        assert res[q]["iters"] == rq["iters"] and res[q]["converged"] == 1
        assert torch.equal(xs[q], xq)
        assert torch.equal(xs2[q], xq) and res2[q]["iters"] == rq["iters"]
    # one problem against the oracle's converged solution
    pr = oracle.Problem(boxes[1])
    xo, _, _ = pr.cg(bh[1], tol=1e-12, max_iter=20000)
    assert rel_norm(to_host(xs[1]), xo) < 1e-4
    batch.close()


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_batch_mixed_equals_solo(geom):
    import torch
    import paper_2108_12188_amd as sem
    say(f"batch mixed geom={geom}")
    boxes, gms = _meshes(sem)
    bs = [gm.rhs(_manufactured(gm), prec=sem.FP64) for gm in gms]
    batch = sem.Batch(gms)
    xs, res = batch.solve(bs, prec=sem.MIXED, geom=geom, tol=1e-8, inner_tol=1e-5)
    for q, gm in enumerate(gms):
        xq, rq = gm.cg_solve(bs[q], prec=sem.MIXED, geom=geom, tol=1e-8, inner_tol=1e-5)
        assert res[q]["converged"] == 1 and rq["converged"] == 1
        assert (res[q]["iters"], res[q]["outer"]) == (rq["iters"], rq["outer"])
        assert torch.equal(xs[q], xq), q
        assert res[q]["rel_res_true"] <= 1e-8
    pr = oracle.Problem(boxes[2])
    bo, _ = pr.rhs_manufactured()           # the oracle's own right-hand side
    assert pr.true_rel_residual(bo, to_host(xs[2])) < 1.1e-8
    # an FP32 solve after the mixed one on the same batch still equals solo
    b32 = [to_dev(random_global_rhs(b, seed=5 + q), torch.float32) for q, b in enumerate(boxes)]
    x32, r32 = batch.solve(b32, prec=sem.FP32, geom=geom, fixed_iters=9)
    for q, gm in enumerate(gms):
        xq, _ = gm.cg_solve(b32[q], prec=sem.FP32, geom=geom, fixed_iters=9)
        assert torch.equal(x32[q], xq), q
    batch.close()


def test_batch_errors():
    import torch
    import paper_2108_12188_amd as sem
    boxes, gms = _meshes(sem)
    with pytest.raises(sem.SemError):
        sem.Batch([gms[0], gms[0]])
    with pytest.raises(sem.SemError) as ei:
        sem.Batch([])
    assert ei.value.code == -1
    batch = sem.Batch(gms[:2])
    bs = [torch.zeros(g.n, dtype=torch.float64, device="cuda") for g in gms[:2]]
    with pytest.raises(ValueError):
        batch.solve(bs[:1], prec=sem.FP32, tol=1e-8)
    with pytest.raises(sem.SemError) as ei:
        batch.solve(bs, prec=sem.FP64, tol=1e-8)
    assert ei.value.code == -6
    batch.close()
