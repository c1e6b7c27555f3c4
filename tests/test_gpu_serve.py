"""Continuous batching on the GPU: requests arriving while others run are
admitted at round boundaries, overlap on the device, every result is
bitwise the one its own solve gives alone, and every served solution meets
the FP64 oracle (its true residual by the oracle's operator, and its distance
to the oracle's own FP64 CG solution of the same problem)."""
import math

import numpy as np
import pytest

from gpu_common import say
from seminputs import box_mesh

pytestmark = pytest.mark.gpu

SPECS = [((3, 3, 2), 5), ((4, 3, 3), 7), ((2, 2, 2), 9), ((5, 4, 3), 5), ((3, 2, 2), 7),
         ((4, 4, 4), 5), ((2, 3, 2), 9), ((3, 3, 3), 7)]


def _forcing(xyz):
    import torch
    return 3 * math.pi ** 2 * torch.sin(math.pi * xyz[0]) * torch.sin(math.pi * xyz[1]) \
        * torch.sin(math.pi * xyz[2])


def _box(tag):
    sh, N = SPECS[tag]
    return box_mesh(*sh, N, perturb=0.1, seed=500 + tag, reorient=True)


def _make_problem(r):
    b = _box(r.tag)
    return b.vert, b.glob_id, b.dirichlet, b.N, _forcing


_ORACLE = {}


def _oracle_solution(tag):
    """The oracle's own manufactured right-hand side and its FP64 CG
    solution to 1e-12 (computed once per mesh)."""
    import oracle
    if tag not in _ORACLE:
        pr = oracle.Problem(_box(tag))
        bo, _ = pr.rhs_manufactured()
        xo, _, _ = pr.cg(bo, tol=1e-12, max_iter=20000, history=False)
        _ORACLE[tag] = (pr, bo, xo)
    return _ORACLE[tag]


def _check_against_oracle(tag, x_dev):
    """Served x against the oracle: true relative residual of the oracle's
    right-hand side with the oracle's operator, and the c-weighted distance to
    the oracle's FP64 solution."""
    pr, bo, xo = _oracle_solution(tag)
    xg = x_dev.detach().cpu().numpy().astype(np.float64)
    rr = pr.true_rel_residual(bo, xg)
    d = xg - xo
    dist = math.sqrt(pr.dot(d, d) / pr.dot(xo, xo))
    assert rr <= 1.1e-8, (tag, rr)
    assert dist <= 1e-6, (tag, dist)
    return rr, dist


@pytest.mark.parametrize("geom", [0, 1], ids=["pre", "otf"])
def test_serving_mix_equals_solo(geom):
    import torch
    import paper_2108_12188_amd as sem
    from paper_2108_12188_amd.serve import GpuEngine, Request, Scheduler, summarize
    say(f"serve geom={geom}")
    reqs = []
    for q, (sh, N) in enumerate(SPECS):
        reqs.append(Request(tag=q, arrival=0.004 * q, n_elem=int(np.prod(sh)), order=N))
    eng = GpuEngine(_make_problem, tol=1e-8, geom=geom, round_iters=8, keep_results=True)
    # a small budget forces queueing: at most ~3 requests resident at once
    budget = 3 * max(eng.footprint(r) for r in reqs)
    sch = Scheduler(eng, budget_bytes=budget, max_slots=4)
    out = sch.run(reqs)
    eng.close()
    st = summarize(out)
    assert st["converged"] == len(reqs), st
    assert sch.peak_used <= budget
    # the device bytes the admitted requests really held (mesh handles plus
    # the caller's tensors, sampled at every round) stayed within the budget
    assert 0 < eng.peak_measured_bytes <= budget, (eng.peak_measured_bytes, budget)
    # overlap: some request was admitted before an earlier one finished
    admits = {t: tm for k, t, tm in sch.log if k == "admit"}
    dones = {t: tm for k, t, tm in sch.log if k == "done"}
    assert any(admits[b] < dones[a] for a in dones for b in admits if b > a)
    for r in out:
        vert, gid, dirichlet, N, forcing = _make_problem(r)
        gm = sem.Mesh(vert, gid, dirichlet, N, g_fp32=(geom == 0))
        b = gm.rhs(forcing(gm.coords()).contiguous(), prec=sem.MIXED)
        x, res = gm.cg_solve(b, prec=sem.MIXED, geom=geom, tol=1e-8)
        assert (res["iters"], res["outer"]) == (r.result["iters"], r.result["outer"])
        assert torch.equal(x, eng.results[r.tag]), r.tag
        assert r.result["rel_res_true"] <= 1e-8
        rr, dist = _check_against_oracle(r.tag, eng.results[r.tag])
        say(f"  request {r.tag}: oracle residual {rr:.2e}, distance to oracle x {dist:.2e}")
        gm.close()


def test_server_reuse_after_release():
    """Requests prepared on a stream of their own (right-hand side and initial
    guess still in flight when they are added) and added after another
    request's mesh was destroyed (its address may be reused): every request
    converges to the bitwise solo result, which meets the oracle."""
    import torch
    import paper_2108_12188_amd as sem
    say("serve reuse, requests prepared on a side stream")
    srv = sem.Server(tol=1e-8, geom=sem.ON_THE_FLY, round_iters=4)
    side = torch.cuda.Stream()
    live = {}

    def add(tag):
        vert, gid, dirichlet, N, forcing = _make_problem(type("R", (), {"tag": tag})())
        gm = sem.Mesh(vert, gid, dirichlet, N, g_fp32=False)
        xyz = gm.coords()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            b = gm.rhs(forcing(xyz).contiguous(), prec=sem.MIXED, stream=side)
            x = torch.zeros_like(b)
            srv.add(gm, b, x, tag, stream=side)
        live[tag] = (gm, b, x)

    results = {}
    add(0)
    add(1)
    nxt = 2
    while live:
        done, _ = srv.step()
        for tag, res in done:
            gm, b, x = live.pop(tag)
            xs, rs = gm.cg_solve(b, prec=sem.MIXED, geom=sem.ON_THE_FLY, tol=1e-8)
            assert res["converged"] == 1, (tag, res)
            assert torch.equal(x, xs), tag
            _check_against_oracle(tag, x)
            results[tag] = res
            gm.close()
            if nxt < len(SPECS):
                add(nxt)
                nxt += 1
    srv.close()
    assert len(results) == len(SPECS)
