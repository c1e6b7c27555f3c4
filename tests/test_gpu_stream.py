"""Non-temporal p and x in the CG-fused operator, chosen when a CG
iteration's vectors, records and edge copy exceed the cache size the
library assumes (sem_set_cache_bytes; 256 MiB, MI355X's Infinity Cache, by
default).  Forcing the choice on small meshes (a 1-byte cache) gives bitwise
the results of plain accesses (a cache larger than any mesh): FP32 at odd
and even orders, both geometric-factor forms, FP64 with G on the fly, and
batches; the streamed solve also follows the FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_common import rel_norm, say, to_dev, to_host
from seminputs import box_mesh, random_global_rhs

pytestmark = pytest.mark.gpu

PLAIN, STREAMED = 1 << 50, 1


@pytest.fixture(autouse=True)
def _default_cache():
    yield
    import paper_2108_12188_amd as sem
    sem.set_cache_bytes(0)


def _both(sem, solve):
    sem.set_cache_bytes(PLAIN)
    a = solve()
    sem.set_cache_bytes(STREAMED)
    b = solve()
    return a, b


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
@pytest.mark.parametrize("N", [5, 6, 7, 9])
def test_fp32_streamed_equals_plain(N, geom):
    import torch
    import paper_2108_12188_amd as sem
    say(f"stream fp32 N={N} geom={geom}")
    mesh = box_mesh(4, 3, 3, N, perturb=0.1, seed=60 + N, permute=True, reorient=True)
    gm = sem.Mesh.from_box(mesh)
    bh = random_global_rhs(mesh, seed=61)
    b = to_dev(bh, torch.float32)
    (x1, r1), (x2, r2) = _both(sem, lambda: gm.cg_solve(b, prec=sem.FP32, geom=geom,
                                                        fixed_iters=15, history=16))
    assert r1["iters"] == r2["iters"] == 15
    assert torch.equal(x1, x2)
    np.testing.assert_array_equal(r1["hist_rho"], r2["hist_rho"])
    pr = oracle.Problem(mesh)
    _, _, hist = pr.cg(bh.astype(np.float32).astype(np.float64), fixed=10)
    np.testing.assert_allclose(r2["hist_rho"][:11], hist["rho"][:11], rtol=1e-4)
    gm.close()


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_fp64_streamed_equals_plain_and_oracle(geom):
    import torch
    import paper_2108_12188_amd as sem
    say(f"stream fp64 geom={geom}")
    mesh = box_mesh(3, 3, 2, 7, perturb=0.1, seed=62, permute=True, reorient=True)
    gm = sem.Mesh.from_box(mesh, g_fp64=True)
    bh = random_global_rhs(mesh, seed=63)
    b = to_dev(bh, torch.float64)
    (x1, r1), (x2, r2) = _both(sem, lambda: gm.cg_solve(b, prec=sem.FP64, geom=geom,
                                                        tol=1e-10, max_iter=2000))
    assert r1["iters"] == r2["iters"] and r2["converged"] == 1
    assert torch.equal(x1, x2)
    xo, _, _ = oracle.Problem(mesh).cg(bh, tol=1e-12, max_iter=5000)
    assert rel_norm(to_host(x2), xo) < 1e-8
    gm.close()


def test_batch_streamed_equals_plain_and_solo():
    import torch
    import paper_2108_12188_amd as sem
    say("stream batch")
    boxes = [box_mesh(3, 3, 2, 7, perturb=0.1, seed=64, permute=True),
             box_mesh(2, 3, 2, 5, perturb=0.1, seed=65, reorient=True),
             box_mesh(2, 2, 2, 9, perturb=0.1, seed=66)]
    gms = [sem.Mesh.from_box(m) for m in boxes]
    bs = [to_dev(random_global_rhs(m, seed=67 + q), torch.float32) for q, m in enumerate(boxes)]
    for geom in (0, 1):
        def solve():
            batch = sem.Batch(gms)
            xs, res = batch.solve(bs, prec=sem.FP32, geom=geom, fixed_iters=13)
            batch.close()
            return xs, res
        (xa, ra), (xb, rb) = _both(sem, solve)
        for q, gm in enumerate(gms):
            assert ra[q]["iters"] == rb[q]["iters"] == 13
            assert torch.equal(xa[q], xb[q]), (geom, q)
            xq, _ = gm.cg_solve(bs[q], prec=sem.FP32, geom=geom, fixed_iters=13)
            assert torch.equal(xb[q], xq), (geom, q)
    for g in gms:
        g.close()


def test_cache_bytes_rejects_negative():
    import paper_2108_12188_amd as sem
    with pytest.raises(sem.SemError):
        sem.set_cache_bytes(-1)
