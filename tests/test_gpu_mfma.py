"""The matrix-core engine of the local operator (FP32, N = 7 and N = 9):
every contraction with D or D^T on the 16-block 4x4x1 MFMA, one element
per workgroup of one (N = 7) or two (N = 9) waves.  It accumulates in the
order of the VALU engine with fused multiply-adds, so its results must be
bitwise those of the VALU engine (operator alone, CG with the fused operator, batches); the VALU
engine itself is held to the oracle by the other operator tests, and the
matrix-core results are also checked against the oracle here."""
import contextlib

import numpy as np
import pytest

import oracle
from gpu_common import oracle_ax_elems, rel_norm, say, to_dev, to_host
from seminputs import box_mesh, random_global_rhs, random_local

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def engine(sem, eng, orders=(7, 9)):
    """Run the block with the operator engine `eng` at the given orders
    (both G forms), restoring the built-in choice after it."""
    for N in orders:
        for g in (sem.PRECOMPUTED, sem.ON_THE_FLY):
            sem.ax_engine_set(N, sem.FP32, g, eng)
    try:
        yield
    finally:
        for N in orders:
            for g in (sem.PRECOMPUTED, sem.ON_THE_FLY):
                sem.ax_engine_set(N, sem.FP32, g, sem.ENGINE_DEFAULT)


def test_engine_selection_and_errors():
    import paper_2108_12188_amd as sem
    with engine(sem, sem.ENGINE_MFMA):
        assert sem.ax_engine_get(7, sem.FP32, sem.ON_THE_FLY) == sem.ENGINE_MFMA
        sh = sem.ax_shape_get(7, sem.FP32, sem.ON_THE_FLY)
        assert sh["elems_per_block"] == 1 and sh["threads"] == 64
        sh = sem.ax_shape_get(9, sem.FP32, sem.ON_THE_FLY)
        assert sh["elems_per_block"] == 1 and sh["threads"] == 128
    with engine(sem, sem.ENGINE_VALU):
        assert sem.ax_engine_get(7, sem.FP32, sem.PRECOMPUTED) == sem.ENGINE_VALU
    # the built-in choice: matrix cores where they time faster than VALU
    for N, g, eng in ((7, sem.PRECOMPUTED, sem.ENGINE_MFMA), (7, sem.ON_THE_FLY, sem.ENGINE_MFMA),
                      (9, sem.ON_THE_FLY, sem.ENGINE_MFMA), (9, sem.PRECOMPUTED, sem.ENGINE_VALU),
                      (5, sem.ON_THE_FLY, sem.ENGINE_VALU)):
        assert sem.ax_engine_get(N, sem.FP32, g) == eng, (N, g)
    assert sem.ax_engine_get(7, sem.FP64, sem.ON_THE_FLY) == sem.ENGINE_VALU
    for N, prec in ((5, sem.FP32), (7, sem.FP64), (9, sem.FP64), (11, sem.FP32)):
        with pytest.raises(sem.SemError) as ei:
            sem.ax_engine_set(N, prec, sem.ON_THE_FLY, sem.ENGINE_MFMA)
        assert ei.value.code == -6
    with pytest.raises(sem.SemError) as ei:
        sem.ax_engine_set(7, sem.FP32, sem.ON_THE_FLY, 5)
    assert ei.value.code == -1


@pytest.mark.parametrize("N", [7, 9])
@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_mfma_operator_bitwise_equals_valu(geom, N):
    """sem_ax on a deformed, permuted, reoriented 5x4x3 mesh (60 elements),
    random and smooth inputs: the two engines agree bit for bit, and both
    meet the FP32 bound against the oracle."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"mfma operator N={N} geom={geom}")
    mesh = box_mesh(5, 4, 3, N, perturb=0.1, seed=71, permute=True, reorient=True)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh)
    x, y, z = pr.coords()
    smooth = np.sin(2.1 * x + 0.3) * np.cos(1.3 * y) * np.exp(0.4 * z)
    for u in (random_local(mesh.n_local, seed=72), smooth):
        u32 = to_dev(u.astype(np.float32), torch.float32)
        with engine(sem, sem.ENGINE_VALU):
            wv = gm.ax(u32, geom=geom)
        with engine(sem, sem.ENGINE_MFMA):
            wm = gm.ax(u32, geom=geom)
        torch.cuda.synchronize()
        assert torch.equal(wv, wm)
        ref = pr.ax_local(u.astype(np.float32).astype(np.float64))
        assert rel_norm(to_host(wm), ref) < 1e-5
    gm.close()


def test_mfma_operator_large_sampled():
    """32^3 elements N = 7 (the full-size operator, 32768 single-wave
    blocks): bitwise equal to the VALU engine everywhere, and 64 sampled
    elements against the oracle one by one."""
    import torch
    import paper_2108_12188_amd as sem
    say("mfma operator 32^3 N=7")
    mesh = box_mesh(32, 32, 32, 7, perturb=0.1, seed=2110)
    gm = sem.Mesh.from_box(mesh)
    u = random_local(mesh.n_local, seed=77).astype(np.float32)
    ud = to_dev(u, torch.float32)
    rng = np.random.default_rng(0)
    elems = np.sort(rng.choice(mesh.E, 64, replace=False))
    elems[-1] = mesh.E - 1
    ref = oracle_ax_elems(mesh, u.astype(np.float64), elems)
    for geom in (0, 1):
        with engine(sem, sem.ENGINE_VALU):
            wv = gm.ax(ud, geom=geom)
        with engine(sem, sem.ENGINE_MFMA):
            wm = gm.ax(ud, geom=geom)
        torch.cuda.synchronize()
        assert torch.equal(wv, wm), geom
        w = to_host(wm).reshape(mesh.E, -1)[elems]
        assert rel_norm(w, ref) < 1e-5, geom
    gm.close()


def test_mfma_cg_large_uneven_grid():
    """28^3 elements N = 7 (21952 elements: more than the fused operator's
    16384 blocks and not a multiple of them, so its blocks walk in launch
    order; the vector grid takes 3659 blocks of three equal grid-stride
    steps): FP32 CG with G on the fly, 8 iterations, bitwise equal between
    the matrix-core and VALU engines; the first rho is <r0, r0, c> of the
    right-hand side in FP64 on the host."""
    import torch
    import paper_2108_12188_amd as sem
    say("mfma cg 28^3 N=7")
    mesh = box_mesh(28, 28, 28, 7, perturb=0.1, seed=2128)
    gm = sem.Mesh.from_box(mesh, g_fp32=False)
    bh = random_global_rhs(mesh, seed=79)
    b = to_dev(bh, torch.float32)
    out = {}
    for eng in (sem.ENGINE_VALU, sem.ENGINE_MFMA):
        with engine(sem, eng):
            out[eng] = gm.cg_solve(b, prec=sem.FP32, geom=1, fixed_iters=8, history=9)
    (xv, rv), (xm, rm) = out[sem.ENGINE_VALU], out[sem.ENGINE_MFMA]
    assert rv["iters"] == rm["iters"] == 8
    assert torch.equal(xv, xm)
    assert np.array_equal(rv["hist_rho"], rm["hist_rho"])
    # rho_0 = <r0, r0, c> for r0 = mask(b) and c = 1/multiplicity, by the
    # oracle's mask, multiplicity and weighted dot (no geometric factors)
    b32 = oracle.mask(mesh.dirichlet, bh.astype(np.float32).astype(np.float64))
    m = oracle.multiplicity(mesh.glob_id, mesh.n_glob)
    np.testing.assert_allclose(rm["hist_rho"][0], oracle.dot(b32, b32, m), rtol=1e-9)
    gm.close()


@pytest.mark.parametrize("N", [7, 9])
@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
@pytest.mark.parametrize("precond", [0, 1], ids=["cg", "jacobi"])
def test_mfma_cg_bitwise_equals_valu(geom, precond, N):
    """FP32 CG (fused operator: p-update, lagged x step, edge copy, alpha
    partials) for 40 fixed iterations: solution and rho history bitwise
    equal between the engines, alpha to FP64 rounding; the first 10
    iterations follow the oracle to 1e-4."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"mfma cg N={N} geom={geom} precond={precond}")
    mesh = box_mesh(6, 5, 4, N, perturb=0.1, seed=73, permute=True, reorient=True)
    gm = sem.Mesh.from_box(mesh)
    b = random_global_rhs(mesh, seed=74)
    bd = to_dev(b, torch.float32)
    out = {}
    for eng in (sem.ENGINE_VALU, sem.ENGINE_MFMA):
        with engine(sem, eng):
            x, r = gm.cg_solve(bd, prec=sem.FP32, geom=geom, fixed_iters=40, history=41,
                               precond=precond)
        out[eng] = (x, r)
    (xv, rv), (xm, rm) = out[sem.ENGINE_VALU], out[sem.ENGINE_MFMA]
    # FP32 vectors and rho are bitwise equal; alpha's denominator sums one
    # FP64 partial per block and the engines use different block counts, so
    # alpha agrees to FP64 rounding (it is rounded to FP32 before use)
    assert torch.equal(xv, xm)
    assert np.array_equal(rv["hist_rho"], rm["hist_rho"])
    np.testing.assert_allclose(rm["hist_alpha"][1:], rv["hist_alpha"][1:], rtol=1e-14)
    pr = oracle.Problem(mesh)
    _, _, hist = pr.pcg(b, fixed=10) if precond else pr.cg(b, fixed=10)
    np.testing.assert_allclose(rm["hist_rho"][:11], hist["rho"][:11], rtol=1e-4)
    gm.close()


def test_mfma_mixed_and_batch():
    """Mixed precision to 1e-10 with the matrix-core inner solve equals the
    VALU one bitwise; a batch of N = 7 and other orders under the
    matrix-core engine equals its solo solves bitwise."""
    import torch
    import paper_2108_12188_amd as sem
    say("mfma mixed + batch")
    mesh = box_mesh(4, 4, 3, 7, perturb=0.1, seed=75, reorient=True)
    gm = sem.Mesh.from_box(mesh)
    b = to_dev(random_global_rhs(mesh, seed=76), torch.float64)
    res = {}
    for eng in (sem.ENGINE_VALU, sem.ENGINE_MFMA):
        with engine(sem, eng):
            res[eng] = gm.cg_solve(b, prec=sem.MIXED, geom=sem.ON_THE_FLY, tol=1e-10)
    assert torch.equal(res[sem.ENGINE_VALU][0], res[sem.ENGINE_MFMA][0])
    assert res[sem.ENGINE_MFMA][1]["converged"] == 1
    gm.close()
    shapes = [((3, 2, 2), 7), ((4, 3, 2), 5), ((2, 3, 2), 9), ((5, 2, 3), 7), ((3, 3, 2), 9)]
    boxes = [box_mesh(*sh, N, perturb=0.1, seed=80 + q, reorient=True, permute=True)
             for q, (sh, N) in enumerate(shapes)]
    gms = [sem.Mesh.from_box(bx) for bx in boxes]
    bs = [to_dev(random_global_rhs(bx, seed=90 + q), torch.float32) for q, bx in enumerate(boxes)]
    with engine(sem, sem.ENGINE_MFMA):
        for geom in (0, 1):
            batch = sem.Batch(gms)
            xs, rs = batch.solve(bs, prec=sem.FP32, geom=geom, fixed_iters=19)
            batch.close()
            for q, g in enumerate(gms):
                xq, rq = g.cg_solve(bs[q], prec=sem.FP32, geom=geom, fixed_iters=19)
                assert rs[q]["iters"] == 19 == rq["iters"]
                assert torch.equal(xs[q], xq), (geom, q)
    for g in gms:
        g.close()


@pytest.mark.parametrize("N", [7, 9])
@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 1, 1), (3, 5, 1)], ids=["E1", "E7", "E15"])
def test_mfma_small_and_odd_meshes(shape, N):
    """One element (a single wave-sized block), and odd element counts: the
    operator and 15 CG iterations bitwise equal to the VALU engine, the CG
    iterates against the oracle."""
    import torch
    import paper_2108_12188_amd as sem
    say(f"mfma small mesh {shape} N={N}")
    mesh = box_mesh(*shape, N, perturb=0.1 if min(shape) > 1 else 0.0, seed=81, reorient=True)
    pr = oracle.Problem(mesh)
    gm = sem.Mesh.from_box(mesh)
    u = to_dev(random_local(mesh.n_local, seed=82).astype(np.float32), torch.float32)
    b = random_global_rhs(mesh, seed=83)
    bd = to_dev(b, torch.float32)
    out = {}
    for eng in (sem.ENGINE_VALU, sem.ENGINE_MFMA):
        with engine(sem, eng):
            w = gm.ax(u, geom=sem.ON_THE_FLY)
            x, r = gm.cg_solve(bd, prec=sem.FP32, geom=sem.ON_THE_FLY, fixed_iters=15,
                               history=16)
        out[eng] = (w, x, r)
    assert torch.equal(out[sem.ENGINE_VALU][0], out[sem.ENGINE_MFMA][0])
    assert torch.equal(out[sem.ENGINE_VALU][1], out[sem.ENGINE_MFMA][1])
    xo, _, hist = pr.cg(b, fixed=15)
    np.testing.assert_allclose(out[sem.ENGINE_MFMA][2]["hist_rho"][:11], hist["rho"][:11],
                               rtol=1e-4)
    gm.close()


def test_mfma_n9_operator_large_sampled():
    """24^3 elements N = 9 (13.8 M points, the mixed-precision workload's
    mesh): bitwise equal to the VALU engine everywhere, and 32 sampled
    elements against the oracle one by one."""
    import torch
    import paper_2108_12188_amd as sem
    say("mfma operator 24^3 N=9")
    mesh = box_mesh(24, 24, 24, 9, perturb=0.1, seed=2111)
    gm = sem.Mesh.from_box(mesh)
    u = random_local(mesh.n_local, seed=78).astype(np.float32)
    ud = to_dev(u, torch.float32)
    rng = np.random.default_rng(1)
    elems = np.sort(rng.choice(mesh.E, 32, replace=False))
    elems[-1] = mesh.E - 1
    ref = oracle_ax_elems(mesh, u.astype(np.float64), elems)
    for geom in (0, 1):
        with engine(sem, sem.ENGINE_VALU):
            wv = gm.ax(ud, geom=geom)
        with engine(sem, sem.ENGINE_MFMA):
            wm = gm.ax(ud, geom=geom)
        torch.cuda.synchronize()
        assert torch.equal(wv, wm), geom
        w = to_host(wm).reshape(mesh.E, -1)[elems]
        assert rel_norm(w, ref) < 1e-5, geom
    gm.close()
