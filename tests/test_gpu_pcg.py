"""Parity of the Jacobi-preconditioned HIP CG (and of the assembled
diagonal it is built from) with the FP64 oracle."""
import dataclasses

import numpy as np
import pytest

import oracle
from gpu_common import rel_norm, say, to_dev, to_host
from seminputs import box_mesh, graded_z, random_global_rhs

pytestmark = pytest.mark.gpu


def _stretched(nx, ny, nz, N, seed):
    """A deformed, permuted, reoriented box graded along z (elements next to
    one face ten times thinner than next to the other), so that the
    diagonal varies strongly and Jacobi changes the iteration."""
    return graded_z(box_mesh(nx, ny, nz, N, perturb=0.1, seed=seed, permute=True,
                             reorient=True), s=3.0)


def test_diag_matches_oracle():
    """sem_diag (element diagonals from the vertices, summed over copies)
    against the oracle's diagonal, on a deformed, permuted mesh of N = 6."""
    import paper_2108_12188_amd as sem
    say("jacobi diagonal 4x3x3 N=6")
    mesh = _stretched(4, 3, 3, 6, seed=17)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh)
    d = to_host(gm.diag())
    do = pr.diag_A()
    np.testing.assert_allclose(d, do, rtol=1e-12)
    # every copy of a global point holds the same sum (bitwise)
    gid = mesh.glob_id.ravel()
    one = np.zeros(mesh.n_glob)
    one[gid] = d
    np.testing.assert_array_equal(d, one[gid])
    gm.close()


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
@pytest.mark.parametrize("graph", [True, False], ids=["graph", "plain"])
def test_pcg_fp64_matches_oracle(geom, graph):
    """FP64 PCG to 1e-9: <r, r, c> and alpha histories, iteration count,
    solution and true residual against the oracle's PCG."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"pcg fp64 geom={geom} graph={graph}")
    mesh = _stretched(4, 4, 3, 5, seed=2108)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh, g_fp64=True, g_fp32=False)
    b = random_global_rhs(mesh, seed=12188)
    xo, it_o, hist = pr.pcg(b, tol=1e-9, max_iter=3000)
    x, res = gm.cg_solve(to_dev(b, torch.float64), prec=sem.FP64, geom=geom, tol=1e-9,
                         max_iter=3000, use_graph=graph, history=40,
                         precond=sem.PRECOND_JACOBI, true_residual=True)
    assert res["converged"] == 1
    assert abs(res["iters"] - it_o) <= 2
    np.testing.assert_allclose(res["hist_rho"][:21], hist["rho"][:21], rtol=1e-10)
    np.testing.assert_allclose(res["hist_alpha"][1:21], hist["alpha"][1:21], rtol=1e-10)
    xg = to_host(x)
    assert rel_norm(xg, xo) < 1e-7
    assert pr.true_rel_residual(b, xg) < 2e-9
    # preconditioning pays on this mesh
    _, it_plain, _ = pr.cg(b, tol=1e-9, max_iter=3000)
    assert res["iters"] < it_plain
    gm.close()


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_pcg_fp32_first_iterations_match_oracle(geom):
    """FP32 PCG, 10 fixed iterations: <r, r, c>, alpha and beta follow the
    FP64 oracle to 1e-4."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"pcg fp32 first iterations geom={geom}")
    mesh = _stretched(6, 5, 4, 7, seed=5)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh)
    b = random_global_rhs(mesh, seed=6)
    xo, _, hist = pr.pcg(b, fixed=10)
    x, res = gm.cg_solve(to_dev(b, torch.float32), prec=sem.FP32, geom=geom, fixed_iters=10,
                         history=12, precond=sem.PRECOND_JACOBI)
    assert res["iters"] == 10
    np.testing.assert_allclose(res["hist_rho"][:11], hist["rho"][:11], rtol=1e-4)
    np.testing.assert_allclose(res["hist_alpha"][1:11], hist["alpha"][1:11], rtol=1e-4)
    assert rel_norm(to_host(x), xo) < 1e-4
    gm.close()


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_pcg_mixed_reaches_1e10(geom):
    """Mixed precision with the preconditioned FP32 inner solve: the true
    FP64 residual reaches 1e-10 and x matches the oracle's PCG solution."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"pcg mixed geom={geom}")
    mesh = _stretched(4, 4, 3, 7, seed=9)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh, g_fp32=True, g_fp64=False)
    b = random_global_rhs(mesh, seed=10)
    x, res = gm.cg_solve(to_dev(b, torch.float64), prec=sem.MIXED, geom=geom, tol=1e-10,
                         inner_tol=1e-5, precond=sem.PRECOND_JACOBI)
    assert res["converged"] == 1 and res["outer"] >= 2
    xh = to_host(x)
    assert pr.true_rel_residual(b, xh) < 1.2e-10
    xs, _, _ = pr.pcg(b, tol=1e-12, max_iter=20000)
    assert rel_norm(xh, xs) < 1e-8
    # the unpreconditioned refinement needs more inner iterations
    _, r0 = gm.cg_solve(to_dev(b, torch.float64), prec=sem.MIXED, geom=geom, tol=1e-10,
                        inner_tol=1e-5)
    assert res["iters"] < r0["iters"]
    gm.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pcg_gather_modes_and_state_reuse(prec):
    """The preconditioned update in both gather modes (conforming mesh:
    sums inside the update; two tied interior nodes: separate pass), and a
    plain solve after a preconditioned one on the same mesh is bitwise the
    plain solve of a fresh mesh."""
    import torch
    import paper_2108_12188_amd as sem
    fp64 = prec == "fp64"
    dt = torch.float64 if fp64 else torch.float32
    mesh = _stretched(3, 2, 2, 4, seed=2111)
    P = mesh.N + 1
    centre = 2 + P * (2 + P * 2)
    gid = mesh.glob_id.copy()
    gid[1, centre] = gid[0, centre]
    tied = dataclasses.replace(mesh, glob_id=gid)
    for m, expect in ((mesh, 1), (tied, 0)):
        say(f"pcg {prec} gather-in-update={expect}")
        pr = oracle.Problem(m)
        gm = sem.Mesh.from_box(m, g_fp64=fp64, g_fp32=not fp64)
        assert gm.info()["gs_in_update"] == expect
        b = random_global_rhs(m, seed=4)
        xo, _, hist = pr.pcg(b, fixed=12)
        x, res = gm.cg_solve(to_dev(b, dt), prec=sem.FP64 if fp64 else sem.FP32,
                             fixed_iters=12, history=13, precond=sem.PRECOND_JACOBI)
        assert res["iters"] == 12
        np.testing.assert_allclose(res["hist_rho"][:13], hist["rho"][:13],
                                   rtol=1e-11 if fp64 else 1e-4)
        np.testing.assert_allclose(res["hist_alpha"][1:13], hist["alpha"][1:13],
                                   rtol=1e-11 if fp64 else 1e-4)
        assert rel_norm(to_host(x), xo) < (1e-11 if fp64 else 1e-4)
        xp, rp = gm.cg_solve(to_dev(b, dt), prec=sem.FP64 if fp64 else sem.FP32, fixed_iters=12)
        gm.close()
        g2 = sem.Mesh.from_box(m, g_fp64=fp64, g_fp32=not fp64)
        xq, rq = g2.cg_solve(to_dev(b, dt), prec=sem.FP64 if fp64 else sem.FP32, fixed_iters=12)
        assert torch.equal(xp, xq)
        g2.close()


def test_pcg_zero_rhs_and_rejections():
    """b = 0 stops at iteration 0 with x = 0; batches and the server take
    no preconditioner; an unknown preconditioner is an argument error."""
    import ctypes as C

    import torch
    import paper_2108_12188_amd as sem
    mesh = box_mesh(2, 2, 2, 3)
    gm = sem.Mesh.from_box(mesh)
    b = torch.zeros(mesh.n_local, dtype=torch.float32, device="cuda")
    x, res = gm.cg_solve(b, prec=sem.FP32, tol=1e-6, precond=sem.PRECOND_JACOBI)
    assert res["iters"] == 0 and res["converged"] == 1
    assert float(x.abs().max()) == 0.0
    with pytest.raises(sem.SemError) as ei:
        gm.cg_solve(b, prec=sem.FP32, tol=1e-6, precond=7)
    assert ei.value.code == -1
    opts = sem.CgOpts(prec=sem.MIXED, geom=0, tol=1e-8, precond=sem.PRECOND_JACOBI)
    srv = C.c_void_p()
    assert sem.lib().sem_server_create(C.byref(opts), 4, C.byref(srv)) == -6
    bt = sem.Batch([gm])
    opts = sem.CgOpts(prec=sem.FP32, geom=0, tol=1e-6, max_iter=10,
                      precond=sem.PRECOND_JACOBI)
    x = torch.zeros_like(b)
    barr = (C.c_void_p * 1)(b.data_ptr())
    xarr = (C.c_void_p * 1)(x.data_ptr())
    res = (sem.CgResult * 1)()
    assert sem.lib().sem_batch_solve(bt._h, C.byref(opts), barr, xarr, res, None) == -6
    bt.close()
    gm.close()
