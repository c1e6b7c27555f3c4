"""sem_dot_noalloc (the weighted inner product without device allocation)
against sem_dot through the C ABI: bitwise equal results on two calls in a
row, the second on a smaller mesh, in FP32 and FP64, and both within FP64
rounding of the oracle's inner product."""
import numpy as np
import pytest

import oracle
from gpu_common import say, to_dev
from seminputs import box_mesh, random_local

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_dot_noalloc_equals_dot(prec):
    import torch
    import paper_2108_12188_amd as sem
    dt = torch.float32 if prec == "fp32" else torch.float64
    # a large mesh (the full 4096 block partials) and then a smaller one
    # (fewer partials: stale ones from the first call must not be summed)
    for case, (shape, N) in enumerate((((16, 16, 12), 7), ((3, 2, 2), 5))):
        say(f"dot_noalloc {prec} call {case}: {shape} N={N}")
        mesh = box_mesh(*shape, N, perturb=0.1, seed=70 + case, reorient=True, permute=True)
        gm = sem.Mesh.from_box(mesh, g_fp32=False)
        a = random_local(mesh.n_local, seed=1 + case)
        b = random_local(mesh.n_local, seed=2 + case)
        if prec == "fp32":
            a = a.astype(np.float32).astype(np.float64)
            b = b.astype(np.float32).astype(np.float64)
        ad, bd = to_dev(a, dt), to_dev(b, dt)
        ref = torch.empty(1, dtype=torch.float64, device="cuda")
        got = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        gm.dot(ad, bd, out=ref)
        gm.dot_noalloc(ad, bd, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (case, float(got), float(ref))
        pr = oracle.Problem(mesh)
        want = pr.dot(a, b)
        assert abs(float(got) - want) <= 1e-12 * pr.dot(np.abs(a), np.abs(b)), (case, want)
        gm.close()
