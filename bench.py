#!/usr/bin/env python3
"""Benchmark of the SEM Poisson CG hot path on one MI355X.

Workload (one step): one FP32 CG solve of 500 fixed iterations (Algorithm 1)
on a 32x32x32 mesh of hexahedra of order N = 7 (16,777,216 local points),
interior vertices perturbed by U(-10%, +10%) of the spacing (seeded), a
random continuous right-hand side U[-1, 1] per global point, homogeneous
Dirichlet boundary.  Every step runs every kernel of the CG iteration:
p-update + local operator + mask + interior <p,w,c>, gather-scatter +
shared <p,w,c> + alpha, x/r update + rho + beta.

Prints ONE JSON line (rank 0) with the throughput in GDOF*iter/s
(local points times iterations per second), the roofline of the dominant
kernel and the FP64 oracle timed on this host as the CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CG GDOF·iter/s + Ax GFLOP/s (% roofline), FP32-mixed vs FP64; p50/p99 solve"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (packed)
FP32_FMA_TFLOPS = 78.6         # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (non-packed FMA)
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ax_bytes_per_point(N: int, geom: str, fused: bool) -> float:
    """Algorithmic FP32 bytes per local point of one operator launch.

    precomputed G: u 4 + G 24 + w 4; on-the-fly G: u 4 + w 4 + 96 B of
    vertices per element.  The CG-fused form also reads r and writes p
    (Algorithm 1 p-update fused into the operator): +8.
    """
    P3 = (N + 1) ** 3
    b = 32.0 if geom == "pre" else 8.0 + 96.0 / P3
    return b + (8.0 if fused else 0.0)


def ax_flops_per_point(N: int, geom: str) -> float:
    """Paper-convention flops per point: 12(N+1)+15 (precomputed G, Eq. 11)
    and 30(N+1)+96 (rematerialized G, Eq. 14 minus the 10 vector flops)."""
    P = N + 1
    return 12.0 * P + 15.0 if geom == "pre" else 30.0 * P + 96.0


def src_hash() -> str:
    h = hashlib.sha256()
    for f in ("sem_ax_order.hip",):
        with open(os.path.join(ROOT, "paper_2108_12188_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_key: str, per_launch_points: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    only if it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "ax_counters.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("src_hash") != src_hash():
        return None
    k = d.get("kernels", {}).get(kernel_key)
    if not k or k.get("n_local") != per_launch_points:
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(mesh, b, budget_s: float = 15.0):
    """FP64 oracle CG on this host's cores, on the same mesh and RHS."""
    import oracle
    t0 = time.perf_counter()
    pr = oracle.Problem(mesh)
    setup = time.perf_counter() - t0
    iters = 2
    t0 = time.perf_counter()
    pr.cg(b, fixed=iters, history=False)
    t = time.perf_counter() - t0
    if t < budget_s / 3:
        iters = max(iters, min(60, int(iters * budget_s / max(t, 1e-3))))
        t0 = time.perf_counter()
        pr.cg(b, fixed=iters, history=False)
        t = time.perf_counter() - t0
    n = mesh.n_local
    return {"value": n * iters / t / 1e9, "unit": "GDOF·iter/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{iters} FP64 CG iterations of the oracle (plus its initial residual) on "
                      f"the same 32^3 N=7 mesh and RHS; {t:.1f} s timed, setup {setup:.1f} s "
                      f"excluded"}


def time_ax(gm, u, geom, reps=50):
    """Median duration (ms) of one sem_ax launch on torch's current stream."""
    import torch
    import paper_2108_12188_amd as sem
    g = sem.PRECOMPUTED if geom == "pre" else sem.ON_THE_FLY
    w = torch.empty_like(u)
    for _ in range(5):
        gm.ax(u, w, geom=g)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, bb in ev:
        a.record()
        gm.ax(u, w, geom=g)
        bb.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(bb) for a, bb in ev)
    return ts[len(ts) // 2]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--geom", choices=["pre", "otf"], default="pre",
                    help="geometric-factor form of the timed solver")
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--nel", type=int, default=32, help="elements per direction")
    ap.add_argument("--order", type=int, default=7)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the operator-alone and FP64 comparison runs")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(independent problems shard trivially, see the design notes)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2108_12188_amd as sem
    from seminputs import MESH_SEED_BASE, RHS_SEED, box_mesh, random_global_rhs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    nel, N, iters = args.nel, args.order, args.iters
    log(f"bench: mesh {nel}^3 N={N}")
    mesh = box_mesh(nel, nel, nel, N, perturb=0.1, seed=MESH_SEED_BASE + 2)
    b_host = random_global_rhs(mesh, seed=RHS_SEED)
    n = mesh.n_local
    gm = sem.Mesh.from_box(mesh, g_fp32=True, g_fp64=False)
    b = torch.as_tensor(b_host.astype(np.float32), device="cuda")
    x = torch.zeros_like(b)
    geom = sem.PRECOMPUTED if args.geom == "pre" else sem.ON_THE_FLY

    def step():
        x.zero_()
        return gm.cg_solve(b, x=x, prec=sem.FP32, geom=geom, fixed_iters=iters)

    log("bench: warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    res = None
    for _ in range(args.steps):
        _, res = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1000.0 * dt / args.steps
    value = n * iters / (dt / args.steps) / 1e9
    log(f"bench: {ms_per_step:.2f} ms/step, {value:.2f} GDOF*iter/s")

    # per-kernel durations of the same solve, timed with HIP events on the
    # solver's stream (no graphs)
    x.zero_()
    _, prof = gm.cg_solve(b, x=x, prec=sem.FP32, geom=geom, fixed_iters=iters,
                          kernel_times=True)
    km = prof["kernel_ms"]
    ax_ms = km["ax"]
    if args.geom == "pre":
        bpp = ax_bytes_per_point(N, "pre", fused=True)
        achieved = bpp * n / (ax_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS}
    else:
        fpp = ax_flops_per_point(N, "otf")
        achieved = fpp * n / (ax_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS}
    roof["kernel"] = "ax_kernel<float, %s, CgFused> (p-update + A_L + mask + <p,w,c> part)" % (
        "precomputed G" if args.geom == "pre" else "on-the-fly G")
    roof["avg_ms"] = ax_ms
    roof["traffic"] = read_traffic(f"cg_fused_{args.geom}_N{N}", n)

    extra = {"kernel_ms": km, "iteration_ms": sum(km.values()),
             "rel_res_recursive": res["rel_res_recursive"] if res else None}
    if not args.no_extras:
        u = torch.as_tensor(np.random.default_rng(1).uniform(-1, 1, n).astype(np.float32),
                            device="cuda")
        for g in ("pre", "otf"):
            ms = time_ax(gm, u, g)
            extra[f"ax_{g}_ms"] = ms
            extra[f"ax_{g}_gbs"] = ax_bytes_per_point(N, g, False) * n / (ms * 1e-3) / 1e9
            extra[f"ax_{g}_gflops_paper"] = ax_flops_per_point(N, g) * n / (ms * 1e-3) / 1e9
        extra["ax_pre_hbm_frac"] = extra["ax_pre_gbs"] / HBM_PEAK_GBS
        extra["ax_otf_fp32_frac"] = extra["ax_otf_gflops_paper"] / 1e3 / FP32_PEAK_TFLOPS
        # the other geometric-factor form through the whole solver
        other = sem.ON_THE_FLY if args.geom == "pre" else sem.PRECOMPUTED
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gm.cg_solve(b, x=x, prec=sem.FP32, geom=other, fixed_iters=iters)
        torch.cuda.synchronize()
        extra["cg_fp32_%s_gdof" % ("otf" if args.geom == "pre" else "pre")] = \
            n * iters / (time.perf_counter() - t1) / 1e9
        # plain FP64 CG on the same mesh (precomputed FP64 G)
        del u
        gm64 = sem.Mesh.from_box(mesh, g_fp32=False, g_fp64=True)
        b64 = torch.as_tensor(b_host, device="cuda")
        x64 = torch.zeros_like(b64)
        it64 = min(iters, 200)
        gm64.cg_solve(b64, x=x64, prec=sem.FP64, fixed_iters=10)
        torch.cuda.synchronize()
        x64.zero_()
        t1 = time.perf_counter()
        gm64.cg_solve(b64, x=x64, prec=sem.FP64, fixed_iters=it64)
        torch.cuda.synchronize()
        extra["cg_fp64_pre_gdof"] = n * it64 / (time.perf_counter() - t1) / 1e9
        gm64.close()
    extra["mesh"] = gm.info()

    cpu = None
    if not args.no_cpu:
        log("bench: oracle CPU baseline")
        cpu = cpu_baseline(mesh, b_host)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GDOF·iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"FP32 CG, {iters} fixed iterations, {nel}^3 hexahedra +-10% "
                               f"deformed (seeded), N={N}, random continuous RHS, Dirichlet box, "
                               f"{'precomputed' if args.geom == 'pre' else 'on-the-fly'} G",
                   "elements": mesh.E, "order": N, "n_local": n, "iterations": iters,
                   "geom": args.geom},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    gm.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
