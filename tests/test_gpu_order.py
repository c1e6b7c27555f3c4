"""Element reordering (sem_element_order: Hilbert, Morton, rows) on an
unstructured-style mesh (shuffled elements, rotated local frames): the
operator on the reordered mesh is bitwise the element-permuted operator of
the input mesh; CG on the reordered mesh matches the oracle on the same
reordered mesh, and the input mesh's solution permuted; the table-free
gather still applies after reordering."""
import dataclasses

import numpy as np
import pytest

import oracle
from gpu_common import rel_norm, say, to_dev, to_host
from seminputs import box_mesh, random_global_rhs, random_local

pytestmark = pytest.mark.gpu


def _meshes(kind):
    import paper_2108_12188_amd as sem
    m = box_mesh(6, 5, 4, 7, perturb=0.1, seed=88, permute=True, reorient=True)
    perm = sem.element_order(m.vert, kind)
    v, gid, d = sem.permute_elements(perm, m.vert, m.glob_id, m.dirichlet)
    r = dataclasses.replace(m, vert=v, glob_id=gid, dirichlet=d)
    return m, r, perm


@pytest.mark.parametrize("kind", [0, 1, 2], ids=["hilbert", "morton", "rows"])
def test_reordered_operator_is_permuted_operator(kind):
    import torch
    import paper_2108_12188_amd as sem
    say(f"order {kind}: operator")
    m, r, perm = _meshes(kind)
    ga = sem.Mesh.from_box(m, g_fp32=True, g_fp64=True)
    gb = sem.Mesh.from_box(r, g_fp32=True, g_fp64=True)
    ia, ib = ga.info(), gb.info()
    for k in ("n_local", "n_glob", "n_shared", "n_groups", "n_dirichlet"):
        assert ia[k] == ib[k], k
    u = random_local(m.n_local, seed=9)
    (ub,) = sem.permute_elements(perm, u)
    for dt in (torch.float32, torch.float64):
        for geom in (sem.PRECOMPUTED, sem.ON_THE_FLY):
            wa = to_host(ga.ax(to_dev(u, dt), geom=geom))
            wb = to_host(gb.ax(to_dev(ub, dt), geom=geom))
            (wap,) = sem.permute_elements(perm, wa)
            np.testing.assert_array_equal(wb, wap)
    ga.close()
    gb.close()


@pytest.mark.parametrize("kind", [0, 1, 2], ids=["hilbert", "morton", "rows"])
def test_reordered_cg_matches_oracle(kind):
    import torch
    import paper_2108_12188_amd as sem
    say(f"order {kind}: CG")
    m, r, perm = _meshes(kind)
    b = random_global_rhs(m, seed=12)
    (bb,) = sem.permute_elements(perm, b)
    pr = oracle.Problem(r)
    xo, _, hist = pr.cg(bb, tol=1e-11, max_iter=5000)
    ga = sem.Mesh.from_box(m, g_fp64=True)
    gb = sem.Mesh.from_box(r, g_fp64=True)
    xa, _ = ga.cg_solve(to_dev(b, torch.float64), prec=sem.FP64, tol=1e-11, max_iter=5000)
    xb, rb = gb.cg_solve(to_dev(bb, torch.float64), prec=sem.FP64, tol=1e-11, max_iter=5000)
    assert rb["converged"] == 1
    (xap,) = sem.permute_elements(perm, to_host(xa))
    assert rel_norm(to_host(xb), xo) < 1e-9
    assert rel_norm(to_host(xb), xap) < 1e-9
    ga.close()
    gb.close()
    # FP32 with the table-free gather forced: first iterations against the
    # oracle on the reordered mesh
    gt = sem.Mesh.from_box(r, table_free=True)
    assert gt.info()["gs_table_free"] == 1
    b32 = bb.astype(np.float32).astype(np.float64)
    _, _, h32 = pr.cg(b32, fixed=10)
    x32, res = gt.cg_solve(to_dev(b32, torch.float32), prec=sem.FP32, geom=sem.ON_THE_FLY,
                           fixed_iters=10, history=11)
    np.testing.assert_allclose(res["hist_rho"][:11], h32["rho"][:11], rtol=1e-4)
    gt.close()
