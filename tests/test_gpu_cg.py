"""Parity of the HIP CG solver (Algorithm 1) and its mixed-precision
refinement with the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
from gpu_common import rel_norm, say, to_dev, to_host
from seminputs import box_mesh, random_global_rhs

pytestmark = pytest.mark.gpu


def _manufactured(gm, pr, prec):
    import torch
    import paper_2108_12188_amd as sem
    xyz = gm.coords()
    f = 3 * math.pi ** 2 * torch.sin(math.pi * xyz[0]) * torch.sin(math.pi * xyz[1]) \
        * torch.sin(math.pi * xyz[2])
    return gm.rhs(f.contiguous(), prec=prec)


@pytest.mark.parametrize("graph", [True, False])
def test_cg_fp64_small_box_matches_oracle(graph):
    """4x4x4 affine elements, N = 7, manufactured forcing, tol 1e-8."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"cg fp64 4^3 N=7 graph={graph}")
    mesh = box_mesh(4, 4, 4, 7)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh, g_fp64=True)
    b = _manufactured(gm, pr, sem.FP64)
    bh = to_host(b)
    bref, u_exact = pr.rhs_manufactured()
    assert rel_norm(bh, bref) < 1e-14
    xo, it_o, hist = pr.cg(bref, tol=1e-8, max_iter=2000)
    x, res = gm.cg_solve(b, prec=sem.FP64, tol=1e-8, max_iter=2000, use_graph=graph,
                         true_residual=True, history=60)
    assert res["converged"] == 1
    assert abs(res["iters"] - it_o) <= 2
    # CG amplifies rounding differences as it converges.  On this problem
    # the oracle against itself, with D, G or b moved by one ulp, keeps rho_i
    # to ~1e-14 relative up to i = 20, then drifts by up to ~20% of rho_i
    # near i = 38 (where rho_i ~ 1e-8 max rho), i.e. by up to ~1.2e-9 of
    # max_j rho_j, while its solution moves by ~5e-12
    # (tests/test_oracle_cg.py::test_cg_history_drift_under_one_ulp_perturbations).
    # So the first 20 iterations must agree tightly, the rest within about
    # four times that drift in absolute terms, and the solution tightly.
    rg, ro = res["hist_rho"], hist["rho"]
    np.testing.assert_allclose(rg[:21], ro[:21], rtol=1e-10)
    np.testing.assert_allclose(res["hist_alpha"][1:21], hist["alpha"][1:21], rtol=1e-10)
    k = min(len(rg), len(ro))
    assert np.max(np.abs(rg[:k] - ro[:k])) <= 5e-9 * np.max(ro)
    xg = to_host(x)
    assert rel_norm(xg, xo) < 1e-10
    assert res["rel_res_true"] < 1.1e-8
    assert pr.true_rel_residual(bref, xg) < 1.1e-8
    assert np.max(np.abs(xg - u_exact)) < 1e-5
    gm.close()


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_cg_fp32_first_iterations_match_oracle(geom):
    """Deformed 6x5x4 mesh, N = 5, random continuous RHS: alpha_i and beta_i of
    the FP32 solver follow the FP64 oracle to 1e-4 for i <= 10."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"cg fp32 first iterations geom={geom}")
    mesh = box_mesh(6, 5, 4, 5, perturb=0.1, seed=2110, permute=True, reorient=True)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh)
    b = random_global_rhs(mesh, seed=12188)
    xo, it_o, hist = pr.cg(b, fixed=10)
    x, res = gm.cg_solve(to_dev(b, torch.float32), prec=sem.FP32, geom=geom, fixed_iters=10,
                         history=12)
    assert res["iters"] == 10
    rho_o, rho_g = hist["rho"][:11], res["hist_rho"][:11]
    np.testing.assert_allclose(rho_g, rho_o, rtol=1e-4)
    np.testing.assert_allclose(res["hist_alpha"][1:11], hist["alpha"][1:11], rtol=1e-4)
    beta_g = rho_g[1:] / rho_g[:-1]
    np.testing.assert_allclose(beta_g, hist["beta"][1:11], rtol=1e-4)
    assert rel_norm(to_host(x), xo) < 1e-4
    gm.close()


def test_cg_deterministic_and_graph_equals_plain():
    import torch
    import paper_2108_12188_amd as sem
    mesh = box_mesh(5, 4, 4, 7, perturb=0.1, seed=4)
    gm = sem.Mesh.from_box(mesh)
    b = to_dev(random_global_rhs(mesh, seed=5), torch.float32)
    x1, r1 = gm.cg_solve(b, prec=sem.FP32, fixed_iters=37, use_graph=True)
    x2, r2 = gm.cg_solve(b, prec=sem.FP32, fixed_iters=37, use_graph=True)
    x3, r3 = gm.cg_solve(b, prec=sem.FP32, fixed_iters=37, use_graph=False, poll_every=5)
    assert torch.equal(x1, x2) and torch.equal(x1, x3)
    assert r1["rel_res_recursive"] == r2["rel_res_recursive"] == r3["rel_res_recursive"]
    gm.close()


def test_cg_zero_rhs_and_nonzero_guess():
    import torch
    import paper_2108_12188_amd as sem
    mesh = box_mesh(3, 3, 3, 4, perturb=0.1, seed=1)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh, g_fp64=True)
    b = torch.zeros(mesh.n_local, dtype=torch.float64, device="cuda")
    x, res = gm.cg_solve(b, prec=sem.FP64, tol=1e-10)
    assert res["iters"] == 0 and res["converged"] == 1
    assert float(x.abs().max()) == 0.0
    # nonzero initial guess: same solution as from zero
    bb = random_global_rhs(mesh, seed=2)
    xg0 = to_dev(np.random.default_rng(0).uniform(-1, 1, mesh.n_local), torch.float64)
    xg0 = to_dev(pr.gs(to_host(xg0)) / pr.m, torch.float64)     # continuous guess
    x1, r1 = gm.cg_solve(to_dev(bb, torch.float64), x=xg0, prec=sem.FP64, tol=1e-11)
    xo, _, _ = pr.cg(bb, tol=1e-12, max_iter=5000)
    assert rel_norm(to_host(x1), xo) < 1e-8
    assert r1["converged"] == 1
    gm.close()


@pytest.mark.parametrize("table_free", [False, True], ids=["table", "table_free"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N,shape,copies", [(2, (1, 1, 1), 1), (1, (2, 2, 2), 8)],
                         ids=["centre", "corner8"])
def test_cg_single_unknown(N, shape, copies, prec, table_free):
    """Meshes with one unknown: the centre of one N = 2 element (no shared
    point), and at N = 1 the middle vertex of a 2x2x2 box, shared by all
    eight elements.  CG (Algorithm 1) reaches the solution in one step."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"cg single unknown N={N} {shape} {prec} table_free={table_free}")
    mesh = box_mesh(*shape, N, perturb=0.1, seed=4)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh, g_fp64=(prec == "fp64"), table_free=table_free)
    bh = random_global_rhs(mesh, seed=5)
    assert np.count_nonzero(bh) == copies
    fp64 = prec == "fp64"
    dt = torch.float64 if fp64 else torch.float32
    x, res = gm.cg_solve(to_dev(bh, dt), prec=sem.FP64 if fp64 else sem.FP32,
                         tol=1e-12 if fp64 else 1e-5, max_iter=50)
    assert res["converged"] == 1 and res["iters"] == 1
    xo, _, _ = pr.cg(bh, tol=1e-14, max_iter=50)
    assert np.count_nonzero(xo) == copies
    assert rel_norm(to_host(x), xo) < (1e-13 if fp64 else 1e-6)
    gm.close()


def test_cg_max_iter_cap():
    import torch
    import paper_2108_12188_amd as sem
    mesh = box_mesh(4, 4, 4, 5, perturb=0.1, seed=3)
    gm = sem.Mesh.from_box(mesh)
    b = to_dev(random_global_rhs(mesh, seed=2), torch.float32)
    x, res = gm.cg_solve(b, prec=sem.FP32, tol=1e-12, max_iter=7)
    assert res["iters"] == 7 and res["converged"] == 0 and res["status"] == 2
    gm.close()


def test_cg_nan_rhs_is_breakdown():
    import torch
    import paper_2108_12188_amd as sem
    mesh = box_mesh(2, 2, 2, 3)
    gm = sem.Mesh.from_box(mesh)
    b = torch.ones(mesh.n_local, dtype=torch.float32, device="cuda")
    b[5] = float("nan")
    x, res = gm.cg_solve(b, prec=sem.FP32, tol=1e-6, max_iter=10)
    assert res["status"] == 3 and res["converged"] == 0
    gm.close()


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_mixed_precision_reaches_1e10(geom):
    """FP32 inner CG + FP64 outer residual: the true FP64 residual (checked
    with the oracle's operator on the returned x) reaches 1e-10."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"mixed geom={geom}")
    mesh = box_mesh(4, 4, 3, 9, perturb=0.1, seed=2111, reorient=True)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh, g_fp32=True, g_fp64=False)
    b = _manufactured(gm, pr, sem.FP64)
    bref, _ = pr.rhs_manufactured()         # the oracle's own right-hand side
    x, res = gm.cg_solve(b, prec=sem.MIXED, geom=geom, tol=1e-10, inner_tol=1e-5)
    assert res["converged"] == 1 and res["outer"] >= 2
    xh = to_host(x)
    assert pr.true_rel_residual(bref, xh) < 1.2e-10
    xs, _, _ = pr.cg(bref, tol=1e-12, max_iter=20000)
    assert rel_norm(xh, xs) < 1e-8
    gm.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cg_gather_in_update_modes(prec):
    """A conforming mesh gathers the shared sums inside the CG update (also
    with a group of 3 copies); a scatter map that ties two element-interior
    nodes (valid, not conforming) takes the separate gather-scatter pass, and
    so does a conforming mesh created with SEM_MESH_GATHER_PASS (the paper's
    schedule).  All follow the oracle."""
    import dataclasses

    import torch
    import paper_2108_12188_amd as sem
    fp64 = prec == "fp64"
    mesh = box_mesh(3, 2, 2, 4, perturb=0.1, seed=2111)
    P = mesh.N + 1
    centre = 2 + P * (2 + P * 2)
    gid = mesh.glob_id.copy()
    gid[1, centre] = gid[0, centre]
    tied = dataclasses.replace(mesh, glob_id=gid)
    # one copy of a face node moved into another face node's group: m = 3
    gid3 = mesh.glob_id.copy()
    gid3[5, P * (2 + P * 2)] = gid3[0, mesh.N + P * (2 + P * 2)]
    odd = dataclasses.replace(mesh, glob_id=gid3)
    for m, expect, kw in ((mesh, 1, {}), (odd, 1, {}), (tied, 0, {}),
                          (mesh, 0, {"gather_pass": True})):
        say(f"cg {prec} gather-in-update={expect} {kw}")
        pr = oracle.Problem(m)
        gm = sem.Mesh.from_box(m, g_fp64=fp64, g_fp32=not fp64, **kw)
        assert gm.info()["gs_in_update"] == expect
        b = random_global_rhs(m, seed=12188)
        xo, _, hist = pr.cg(b, fixed=12)
        x, res = gm.cg_solve(to_dev(b, torch.float64 if fp64 else torch.float32),
                             prec=sem.FP64 if fp64 else sem.FP32, fixed_iters=12, history=13)
        assert res["iters"] == 12
        np.testing.assert_allclose(res["hist_rho"][:13], hist["rho"][:13],
                                   rtol=1e-11 if fp64 else 1e-4)
        assert rel_norm(to_host(x), xo) < (1e-11 if fp64 else 1e-4)
        gm.close()


@pytest.mark.parametrize("N", [5, 7, 9])
def test_cg_table_free_gather_bitwise_equals_table(N):
    """Odd orders can gather the shared sums in the update from each point's
    position and per-element face and edge records instead of a per-point
    table (forced here with SEM_MESH_GATHER_TABLE_FREE: these meshes are
    below the size from which it is the default): FP32 (both G forms, with
    and without Jacobi), FP64 and mixed solves give bitwise the results of
    the table form (SEM_MESH_GATHER_TABLE) on a permuted, reoriented mesh,
    and on one whose only Dirichlet face is x = 0 (free boundary faces,
    edges and corners)."""
    import dataclasses

    import torch
    import paper_2108_12188_amd as sem
    base = box_mesh(4, 3, 3, N, perturb=0.1, seed=90 + N, permute=True, reorient=True)
    GX = 4 * N + 1
    one_face = dataclasses.replace(base, dirichlet=(base.glob_id % GX == 0).astype(np.uint8))
    for mesh, tag in ((base, "box"), (one_face, "x0")):
        b = random_global_rhs(mesh, seed=91)
        meshes = [sem.Mesh.from_box(mesh, g_fp32=True, g_fp64=True, table_free=True),
                  sem.Mesh.from_box(mesh, g_fp32=True, g_fp64=True, gather_table=True)]
        assert meshes[0].info()["gs_table_free"] == 1
        assert meshes[1].info()["gs_table_free"] == 0
        runs = [("fp32-otf", sem.FP32, sem.ON_THE_FLY, 0), ("fp32-otf-jacobi", sem.FP32,
                                                          sem.ON_THE_FLY, 1),
                ("fp32-pre", sem.FP32, sem.PRECOMPUTED, 0), ("fp64-pre", sem.FP64,
                                                              sem.PRECOMPUTED, 0)]
        for name, prec, geom, pc in runs:
            say(f"table-free gather N={N} {tag} {name}")
            out = []
            for gm in meshes:
                dt = torch.float64 if prec == sem.FP64 else torch.float32
                x, r = gm.cg_solve(to_dev(b, dt), prec=prec, geom=geom, fixed_iters=30,
                                   history=31, precond=pc)
                out.append((to_host(x), r))
            (x0, r0), (x1, r1) = out
            assert np.array_equal(x0, x1), name
            assert np.array_equal(r0["hist_rho"], r1["hist_rho"]), name
            # alpha_i from i = 1 (entry 0 is not written)
            assert np.array_equal(r0["hist_alpha"][1:], r1["hist_alpha"][1:]), name
        say(f"table-free gather N={N} {tag} mixed")
        out = [gm.cg_solve(to_dev(b, torch.float64), prec=sem.MIXED, geom=sem.ON_THE_FLY,
                           tol=1e-10) for gm in meshes]
        assert out[0][1]["iters"] == out[1][1]["iters"]
        assert np.array_equal(to_host(out[0][0]), to_host(out[1][0]))
        for gm in meshes:
            gm.close()
    # an even order keeps the table, even when asked
    even = sem.Mesh.from_box(box_mesh(2, 2, 2, 6, perturb=0.1, seed=92), table_free=True)
    assert even.info()["gs_table_free"] == 0 and even.info()["gs_in_update"] == 1
    even.close()


def test_gather_form_default_by_size_and_flags():
    """The table-free gather is the default from 2^19 local points on
    (24^3 N = 7: 7.1 M points; 8^3 N = 7, 262144 points, keeps the table),
    the table below (small meshes run faster with it); asking for both
    forms is an error."""
    import paper_2108_12188_amd as sem
    small = box_mesh(3, 3, 3, 7, perturb=0.1, seed=93)
    gm = sem.Mesh.from_box(small)
    assert gm.info()["gs_table_free"] == 0
    gm.close()
    # the boundary: 8 x 8 x 15 elements (491520 points) keep the table,
    # 8 x 8 x 16 (524288 = 2^19 points) take the table-free form
    for nz, want in ((15, 0), (16, 1)):
        gm = sem.Mesh.from_box(box_mesh(8, 8, nz, 7, perturb=0.1, seed=96), g_fp32=False)
        assert gm.info()["gs_table_free"] == want
        gm.close()
    with pytest.raises(sem.SemError) as ei:
        sem.Mesh.from_box(small, gather_table=True, table_free=True)
    assert ei.value.code == -1
    say("gather form default on 24^3 N=7")
    import torch
    box = box_mesh(24, 24, 24, 7, perturb=0.1, seed=94)
    big = sem.Mesh.from_box(box, g_fp32=False)
    assert big.info()["gs_table_free"] == 1
    # at this size too the two forms agree bitwise (10 FP32 iterations)
    b = to_dev(random_global_rhs(box, seed=95), torch.float32)
    x0, r0 = big.cg_solve(b, prec=sem.FP32, geom=sem.ON_THE_FLY, fixed_iters=10, history=11)
    big.close()
    tab = sem.Mesh.from_box(box, g_fp32=False, gather_table=True)
    assert tab.info()["gs_table_free"] == 0
    x1, r1 = tab.cg_solve(b, prec=sem.FP32, geom=sem.ON_THE_FLY, fixed_iters=10, history=11)
    tab.close()
    assert torch.equal(x0, x1)
    assert np.array_equal(r0["hist_rho"], r1["hist_rho"])


def test_cg_fp32_full_size_matches_oracle():
    """The headline workload in the launch configuration the benchmark times
    (32^3 hexahedra, N = 7, +-10% deformed, its mesh and RHS seeds, FP32,
    on-the-fly G, the built-in engine and gather form: matrix cores,
    table-free gather): the first 10 iterations against the FP64 oracle,
    rho to 1e-4 and x to 1e-4 normwise."""
    import torch
    import paper_2108_12188_amd as sem
    from seminputs import MESH_SEED_BASE, RHS_SEED
    say("cg fp32 full size 32^3 N=7 vs oracle")
    mesh = box_mesh(32, 32, 32, 7, perturb=0.1, seed=MESH_SEED_BASE + 2)
    b = random_global_rhs(mesh, seed=RHS_SEED)
    gm = sem.Mesh.from_box(mesh)
    assert gm.info()["gs_table_free"] == 1
    assert sem.ax_engine_get(7, sem.FP32, sem.ON_THE_FLY) == sem.ENGINE_MFMA
    x, res = gm.cg_solve(to_dev(b, torch.float32), prec=sem.FP32, geom=sem.ON_THE_FLY,
                         fixed_iters=10, history=11)
    xh = to_host(x)
    gm.close()
    del x
    pr = oracle.Problem(mesh)
    xo, _, hist = pr.cg(b, fixed=10)
    np.testing.assert_allclose(res["hist_rho"][:11], hist["rho"][:11], rtol=1e-4)
    assert rel_norm(xh, xo) < 1e-4
