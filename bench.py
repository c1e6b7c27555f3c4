#!/usr/bin/env python3
"""Benchmark of the SEM Poisson CG hot path on one MI355X.

Workload (one step): one FP32 CG solve of 500 fixed iterations (Algorithm 1)
on a 32x32x32 mesh of hexahedra of order N = 7 (16,777,216 local points),
interior vertices perturbed by U(-10%, +10%) of the spacing (seeded), a
random continuous right-hand side U[-1, 1] per global point, homogeneous
Dirichlet boundary.  Every step runs every kernel of the CG iteration:
p-update + previous x step + local operator + <p,w,c> partials; sums of the
edge and vertex groups + alpha; gather of the face pairs + mask + r update +
rho + beta; and the closing x step.

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
CLOCK_HZ = 2.4e9               # MI355X engine clock (256 CUs x 4 SIMDs)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ax_bytes_per_point(N: int, geom: str, fused: bool) -> float:
    """Algorithmic FP32 bytes per local point of one operator launch.

    precomputed G: u 4 + G 24 + w 4; on-the-fly G: u 4 + w 4 + 96 B of
    vertices per element.  The CG-fused form (u = p_old) also reads r and
    writes p (the p-update), reads and writes x (the previous iteration's x
    step) and writes the compact copy of the 12N - 4 edge and corner nodes of
    every element: +16 + 4 (12N - 4) / P^3.
    """
    P3 = (N + 1) ** 3
    b = 32.0 if geom == "pre" else 8.0 + 96.0 / P3
    return b + (16.0 + 4.0 * (12 * N - 4) / P3 if fused else 0.0)


def update_bytes_per_point(N: int, shared_frac: float, jacobi: bool = False,
                           table_free: bool = True) -> float:
    """Algorithmic FP32 bytes per local point of the update with gather: r
    read and written 8, w 4, one gathered value per shared point, and the
    gather's description: with the table-free form the element's 8-byte
    face and edge-slot records, 8 (6 + 12N - 4) / P^3; with the per-point
    table a 4-byte entry and a 1-byte code per point.  With the Jacobi
    preconditioner also M^-1 read and z written (+8)."""
    P3 = (N + 1) ** 3
    desc = 8.0 * (6 + 12 * N - 4) / P3 if table_free else 5.0
    return 8.0 + 4.0 + 4.0 * shared_frac + desc + (8.0 if jacobi else 0.0)


def ax_flops_per_point(N: int, geom: str) -> float:
    """Paper-convention flops per point: 12(N+1)+15 (precomputed G, Eq. 11)
    and 30(N+1)+96 (rematerialized G, Eq. 14 minus the 10 vector flops)."""
    P = N + 1
    return 12.0 * P + 15.0 if geom == "pre" else 30.0 * P + 96.0


# the sources of every kernel the committed counter summary describes (the
# operator, the gathered update and its group sums, the stand-alone
# gather-scatter)
COUNTER_SOURCES = ("sem_ax_order.hip", "sem_vec.hip", "sem_vec_body.h", "sem_gs.hip",
                   "sem_gs_body.h")


def src_hash() -> str:
    h = hashlib.sha256()
    for f in COUNTER_SOURCES:
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


def read_counters(key: str, per_launch_points: int):
    """One kernel's entry of the committed rocprofv3 counter summary
    (profiles/ax_counters.json), only if it was taken on the current kernel
    source and at this size; else None."""
    p = os.path.join(ROOT, "profiles", "ax_counters.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("src_hash") != src_hash():
        return None
    k = d.get("kernels", {}).get(key)
    if not k or k.get("n_local") != per_launch_points:
        return None
    return k


def otf_executed(ms: float, n: int, N: int):
    """Executed work of the stand-alone on-the-fly operator against the
    units that could bind it, from its committed instruction counters
    (SQ_INSTS_VALU, SQ_INSTS_MFMA, SQ_VALU_MFMA_BUSY_CYCLES per launch) and
    the duration `ms` measured in this run: the fraction of the VALU issue
    rate (1024 SIMDs, one wave64 instruction per 4 cycles: 78.6 TFLOP/s of
    non-packed FP32 FMAs), of the matrix cores' time, and of HBM."""
    k = read_counters(f"ax_otf_plain_N{N}", n)
    if not k:
        return None
    t = ms * 1e-3
    simd_cycles = 1024 * CLOCK_HZ * t
    E = n // (N + 1) ** 3
    out = {"valu_insts_per_element": k["valu_insts_per_launch"] / E,
           "mfma_insts_per_element": k["mfma_insts_per_launch"] / E,
           "executed_flop_per_point": k.get("executed_flop_per_point"),
           "paper_flop_per_point": ax_flops_per_point(N, "otf"),
           "valu_issue_frac": 4 * k["valu_insts_per_launch"] / simd_cycles,
           "mfma_busy_frac": k["mfma_busy_cycles_per_launch"] / simd_cycles,
           "hbm_frac": k["hbm_bytes_per_launch"] / t / (HBM_PEAK_GBS * 1e9),
           "source": "profiles/ax_counters.json (rocprofv3 --pmc of bench.py --ax-only, same "
                     "kernel source, hash-checked); duration from this run"}
    out["executed_tflops"] = (out["executed_flop_per_point"] or 0) * n / t / 1e12
    units = {"VALU issue (non-packed FP32, 78.6 TFLOP/s of FMAs)": out["valu_issue_frac"],
             "matrix cores": out["mfma_busy_frac"], "HBM": out["hbm_frac"]}
    out["binding_unit"] = max(units, key=units.get)
    out["frac_of_binding_unit"] = units[out["binding_unit"]]
    return out


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
    cores = oracle.num_threads()
    # the same solve on one host thread, 2 iterations (the oracle's results
    # do not depend on its thread count)
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        pr.cg(b, fixed=2, history=False)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    return {"value": n * iters / t / 1e9, "unit": "GDOF·iter/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{iters} FP64 CG iterations of the oracle (plus its initial residual) on "
                      f"the same 32^3 N=7 mesh and RHS; {t:.1f} s timed, setup {setup:.1f} s "
                      f"excluded",
            "one_thread_value": n * 2 / t1 / 1e9,
            "one_thread_sample": f"2 iterations (plus the initial residual) on 1 thread, "
                                 f"{t1:.1f} s",
            "host": host_cpu()}


def host_cpu():
    """CPU model and the logical CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def bench_references() -> dict:
    """FP64 oracle values for the large workloads, written by
    tests/golden/make_bench_references.py (empty if absent)."""
    p = os.path.join(ROOT, "tests", "golden", "bench_references.json")
    try:
        with open(p) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def fp64_latency(geom, solves=50):
    """Plain FP64 CG on 4^3 affine hexahedra, N = 7, manufactured forcing,
    tol 1e-8: p50/p99 over `solves` solves and time per iteration."""
    import torch

    import paper_2108_12188_amd as sem
    from seminputs import box_mesh
    gm = sem.Mesh.from_box(box_mesh(4, 4, 4, 7), g_fp32=False, g_fp64=True)
    xyz = gm.coords()
    b = gm.rhs(_forcing(xyz), prec=sem.FP64)
    for _ in range(5):
        gm.cg_solve(b, prec=sem.FP64, geom=geom, tol=1e-8)
    torch.cuda.synchronize()
    times, res = [], None
    for _ in range(solves):
        t0 = time.perf_counter()
        _, res = gm.cg_solve(b, prec=sem.FP64, geom=geom, tol=1e-8)
        times.append(time.perf_counter() - t0)
    x, rt = gm.cg_solve(b, prec=sem.FP64, geom=geom, tol=1e-8, true_residual=True)
    err = float((x - _exact(xyz)).abs().max())
    gm.close()
    p50 = _pct(times, 50)
    return {"p50_ms": p50 * 1e3, "p99_ms": _pct(times, 99) * 1e3, "solves": solves,
            "iters": res["iters"], "us_per_iter": p50 / res["iters"] * 1e6,
            "rel_res_true": rt["rel_res_true"], "max_err_vs_exact_u": err}


def mixed_vs_fp64(ref=None):
    """24^3 deformed hexahedra, N = 9, manufactured forcing: mixed precision
    (FP32 inner CG with G on the fly, FP64 outer residual) against plain FP64
    CG (precomputed FP64 G), both to a true relative residual of 1e-10.  With
    `ref` (the oracle's FP64 solution to 1e-12 at sampled points) the
    sampled error of both solutions against it."""
    import numpy as np
    import torch

    import paper_2108_12188_amd as sem
    from seminputs import MESH_SEED_BASE, box_mesh
    mesh = box_mesh(24, 24, 24, 9, perturb=0.1, seed=MESH_SEED_BASE + 3)
    gm = sem.Mesh.from_box(mesh, g_fp32=False, g_fp64=True)
    n = mesh.n_local
    xyz = gm.coords()
    b = gm.rhs(_forcing(xyz), prec=sem.FP64)
    u = _exact(xyz)
    del xyz
    idx = None
    if ref:
        idx = torch.as_tensor(np.asarray(ref["sample_index"], dtype=np.int64), device="cuda")
        xs = np.asarray(ref["sample_x"])
    out = {}
    for label, prec, geom in (("mixed", sem.MIXED, sem.ON_THE_FLY),
                              ("fp64", sem.FP64, sem.PRECOMPUTED)):
        gm.cg_solve(b, prec=prec, geom=geom, tol=1e-3, max_iter=50)      # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, r = gm.cg_solve(b, prec=prec, geom=geom, tol=1e-10, max_iter=100000,
                           true_residual=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        row = {"seconds": dt, "iters": r["iters"], "outer": r["outer"],
               "rel_res_true": r["rel_res_true"], "converged": r["converged"],
               "gdof_iter_per_s": n * r["iters"] / dt / 1e9,
               "max_err_vs_exact_u": float((x - u).abs().max())}
        if idx is not None:
            got = x[idx].cpu().numpy()
            row["sampled_max_rel_err_vs_oracle_xstar"] = float(
                np.max(np.abs(got - xs)) / np.max(np.abs(xs)))
        out[label] = row
        del x
    gm.close()
    out["speedup_mixed_vs_fp64"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    if ref:
        out["oracle_xstar"] = {"tol": ref["tol"], "iterations": ref["iterations"],
                               "samples": len(ref["sample_index"]),
                               "source": "tests/golden/bench_references.json"}
    return out


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
    ap.add_argument("--geom", choices=["pre", "otf"], default="otf",
                    help="geometric-factor form of the timed solver")
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4, 5, 6, 7, 8, 9],
                    help="2: the headline FP32 CG throughput line; 1, 3, 4, 5: the other "
                         "workloads (FP64 latency, mixed vs FP64, batched, serving); "
                         "6: Jacobi-preconditioned CG against plain CG; 7: FP32 CG "
                         "throughput against the element count; 8: the headline CG on "
                         "unstructured element numberings, reordered or not; 9: the paper's "
                         "performance model (Eq. 15, Table 2) on this GPU")
    ap.add_argument("--requests", type=int, default=2000, help="serving: number of requests")
    ap.add_argument("--rate", type=float, default=0.0, help="serving: arrivals per second "
                    "(0: 0.8 x the measured batched capacity)")
    ap.add_argument("--round-iters", type=int, default=32,
                    help="serving: CG iterations of the running requests per server round")
    ap.add_argument("--slots", type=int, default=128,
                    help="serving: requests admitted at once at most (and the device budget)")
    ap.add_argument("--no-tune", action="store_true", help="ignore the tuned tile shapes")
    ap.add_argument("--engine", choices=["default", "valu", "mfma"], default="default",
                    help="contraction engine of the FP32 local operator at the bench order")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 256 MiB device-to-device copy (reference kernel of known "
                         "size for HBM counter calibration)")
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--nel", type=int, default=32, help="elements per direction")
    ap.add_argument("--order", type=int, default=7)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the operator-alone and FP64 comparison runs")
    ap.add_argument("--ax-only", action="store_true",
                    help="time only the local operator alone (precomputed and on-the-fly G, "
                         "50 launches each) on the bench mesh and print their durations "
                         "(for counter profiles)")
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
    if not args.no_tune:
        from paper_2108_12188_amd import tune
        log(f"bench: {tune.apply()} tuned tile shapes applied")
    if args.engine != "default":
        eng = sem.ENGINE_VALU if args.engine == "valu" else sem.ENGINE_MFMA
        for g in (sem.PRECOMPUTED, sem.ON_THE_FLY):
            sem.ax_engine_set(args.order, sem.FP32, g, eng)
        log(f"bench: operator engine {args.engine} at N={args.order}")
    if args.config != 2:
        return SUITES[args.config](args)
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

    if args.copy_calib:
        ca = torch.empty(64 << 20, dtype=torch.float32, device="cuda").uniform_()
        cb = torch.empty_like(ca)
        for _ in range(3):
            cb.copy_(ca)
        torch.cuda.synchronize()
        del ca, cb
    if args.ax_only:
        u = torch.as_tensor(np.random.default_rng(1).uniform(-1, 1, n).astype(np.float32),
                            device="cuda")
        ms = {g: time_ax(gm, u, g) for g in ("pre", "otf")}
        # the stand-alone gather-scatter (in place, with the mask) in FP32
        # and FP64, on a fresh copy of u before every timed launch
        gs_ms = {}
        for name, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
            src = u.to(dt)
            w = torch.empty_like(src)
            ts = []
            for rep in range(55):
                w.copy_(src)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                gm.gs(w, mask=True)
                e1.record()
                if rep >= 5:
                    ts.append((e0, e1))
            torch.cuda.synchronize()
            gs_ms[name] = sorted(a.elapsed_time(b_) for a, b_ in ts)[len(ts) // 2]
        info = gm.info()
        return _emit({"metric": "local operator and gather-scatter alone, median of 50 launches",
                      "ax_pre_ms": ms["pre"], "ax_otf_ms": ms["otf"],
                      "gs_fp32_ms": gs_ms["fp32"], "gs_fp64_ms": gs_ms["fp64"],
                      "n_local": n, "n_shared": info["n_shared"],
                      "config": {"workload": f"{nel}^3 N={N} +-10% deformed, FP32"}})

    log("bench: warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    res, timed = None, []
    for _ in range(args.steps):
        _, res = step()
        timed.append(res)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # every timed solve must have run all its iterations (status 2: the
    # fixed count was reached; a breakdown, status 3, would stop early)
    for r in timed:
        if r["iters"] != iters or r["status"] != 2:
            raise RuntimeError(f"a timed solve stopped early: {r}")
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
    # The CG-fused operator moves 24.8 (on-the-fly G) or 48.6 (precomputed G)
    # algorithmic bytes per point for 30P+96 or 12P+15 paper-convention flops:
    # both intensities lie below the FP32 machine balance (157.3 TFLOP/s over
    # 8 TB/s = 19.7 flop/B), so HBM bounds either form.
    bpp = ax_bytes_per_point(N, args.geom, fused=True)
    achieved = bpp * n / (ax_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS}
    roof["flops_tflops_paper"] = ax_flops_per_point(N, args.geom) * n / (ax_ms * 1e-3) / 1e12
    mfma = sem.ax_engine_get(N, sem.FP32, geom) == sem.ENGINE_MFMA
    roof["kernel"] = "%s<%s, CgFused> (p-update + previous x step + A_L + <p,w,c> partials)" % (
        "ax_mfma_kernel" if mfma else "ax_kernel<float>",
        "precomputed G" if args.geom == "pre" else "on-the-fly G")
    roof["engine"] = "mfma" if mfma else "valu"
    if mfma:
        # the six D / D^T contractions on the 4x4x1 MFMA: 96 instructions of
        # 512 flops per element
        E = n // (N + 1) ** 3
        roof["mfma_tflops"] = 96 * 512 * E / (ax_ms * 1e-3) / 1e12
        roof["mfma_frac"] = roof["mfma_tflops"] / FP32_PEAK_TFLOPS
    roof["avg_ms"] = ax_ms
    roof["traffic"] = read_traffic(f"cg_fused_{args.geom}_N{N}", n)
    roof["traffic_source"] = (
        "profiles/ax_counters.json: rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, of this "
        "workload on the same kernel source (hash-checked), calibrated against a 256 MiB "
        "copy; not measured in this run" if roof["traffic"] is not None else
        "none recorded for the current kernel source")

    info = gm.info()
    extra = {"gather_form": "table-free" if info["gs_table_free"] else
             ("per-point table" if info["gs_in_update"] else "gather-scatter pass"),
             "kernel_ms": km, "iteration_ms": sum(km.values()),
             "timed_solves": {"count": len(timed), "iterations_each": iters,
                              "status_each": sorted({r["status"] for r in timed})},
             "rel_res_recursive": res["rel_res_recursive"] if res else None}
    # the FP64 true residual of the FP32 iterate after the 500 iterations,
    # beside the FP64 oracle's after the same iterations (committed
    # reference values written by tests/golden/make_bench_references.py)
    x.zero_()
    _, rt = gm.cg_solve(b, x=x, prec=sem.FP32, geom=geom, fixed_iters=iters, true_residual=True)
    extra["rel_res_true_fp64"] = rt["rel_res_true"]
    refs = bench_references()
    hl = refs.get("headline") if (nel, N, iters) == (32, 7, 500) else None
    if hl:
        extra["oracle_fp64_after_same_iterations"] = {
            "rel_res_true": hl["rel_res_true"], "rel_res_recursive": hl["rel_res_recursive"],
            "source": "tests/golden/bench_references.json (FP64 oracle, 500 iterations)"}
    if not args.no_extras:
        u = torch.as_tensor(np.random.default_rng(1).uniform(-1, 1, n).astype(np.float32),
                            device="cuda")
        for g in ("pre", "otf"):
            ms = time_ax(gm, u, g)
            extra[f"ax_{g}_ms"] = ms
            extra[f"ax_{g}_gbs"] = ax_bytes_per_point(N, g, False) * n / (ms * 1e-3) / 1e9
            extra[f"ax_{g}_gflops_paper"] = ax_flops_per_point(N, g) * n / (ms * 1e-3) / 1e9
        extra["ax_pre_hbm_frac"] = extra["ax_pre_gbs"] / HBM_PEAK_GBS
        # paper-convention flops (30P+96 per point) over the packed FP32
        # peak: a convention, not what runs (the D contractions run on the
        # matrix cores, the geometry on the non-packed VALU)
        extra["ax_otf_fp32_frac_paper_convention"] = \
            extra["ax_otf_gflops_paper"] / 1e3 / FP32_PEAK_TFLOPS
        extra["ax_otf_executed"] = otf_executed(extra["ax_otf_ms"], n, N)
        # the other geometric-factor form through the whole solver
        other = sem.ON_THE_FLY if args.geom == "pre" else sem.PRECOMPUTED
        x.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gm.cg_solve(b, x=x, prec=sem.FP32, geom=other, fixed_iters=iters)
        torch.cuda.synchronize()
        extra["cg_fp32_%s_gdof" % ("otf" if args.geom == "pre" else "pre")] = \
            n * iters / (time.perf_counter() - t1) / 1e9
        # the same fused operator on the other contraction engine (the
        # choice rests on this comparison at this order)
        if mfma:
            sem.ax_engine_set(N, sem.FP32, geom, sem.ENGINE_VALU)
            x.zero_()
            _, pv = gm.cg_solve(b, x=x, prec=sem.FP32, geom=geom, fixed_iters=min(iters, 200),
                                kernel_times=True)
            sem.ax_engine_set(N, sem.FP32, geom, sem.ENGINE_DEFAULT)
            extra["ax_fused_valu_engine_ms"] = pv["kernel_ms"]["ax"]
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
        del b64, x64
        log("bench: FP64 latency (4^3 N=7) and mixed vs FP64 to 1e-10 (24^3 N=9)")
        extra["fp64_latency_4cube_N7"] = fp64_latency(geom)
        extra["mixed_vs_fp64_24cube_N9"] = mixed_vs_fp64(refs.get("mixed_24_N9"))
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


# ---------------------------------------------------------------------------
# The other workloads (each prints one JSON line of its own)
# ---------------------------------------------------------------------------
def _forcing(xyz):
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) (manufactured u = sin sin sin)."""
    import torch
    return (3 * math.pi ** 2 * torch.sin(math.pi * xyz[0]) * torch.sin(math.pi * xyz[1])
            * torch.sin(math.pi * xyz[2])).contiguous()


def _exact(xyz):
    import torch
    return torch.sin(math.pi * xyz[0]) * torch.sin(math.pi * xyz[1]) * torch.sin(math.pi * xyz[2])


def _pct(v, p):
    v = sorted(v)
    k = min(len(v) - 1, max(0, int(math.ceil(p / 100.0 * len(v))) - 1))
    return v[k]


def _emit(d):
    print(json.dumps(d), flush=True)
    return 0


def run_config1(args):
    """Plain FP64 CG, 4^3 affine elements, N = 7, manufactured forcing, 1e-8:
    latency per solve (p50/p99 over 50 solves) and per iteration."""
    import numpy as np
    import torch

    import oracle
    import paper_2108_12188_amd as sem
    from seminputs import box_mesh
    mesh = box_mesh(4, 4, 4, 7)
    gm = sem.Mesh.from_box(mesh, g_fp32=False, g_fp64=True)
    xyz = gm.coords()
    b = gm.rhs(_forcing(xyz), prec=sem.FP64)
    geom = sem.PRECOMPUTED if args.geom == "pre" else sem.ON_THE_FLY
    for _ in range(5):
        gm.cg_solve(b, prec=sem.FP64, geom=geom, tol=1e-8)
    torch.cuda.synchronize()
    times, res = [], None
    for _ in range(50):
        t0 = time.perf_counter()
        x, res = gm.cg_solve(b, prec=sem.FP64, geom=geom, tol=1e-8)
        times.append(time.perf_counter() - t0)
    x, res_t = gm.cg_solve(b, prec=sem.FP64, geom=geom, tol=1e-8, true_residual=True)
    err = float((x - _exact(xyz)).abs().max())
    pr = oracle.Problem(mesh)
    bo, _ = pr.rhs_manufactured()       # the oracle's own right-hand side
    t0 = time.perf_counter()
    xo, it_o, _ = pr.cg(bo, tol=1e-8, max_iter=5000, history=False)
    t_cpu = time.perf_counter() - t0
    xd = float(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
    p50 = _pct(times, 50)
    return _emit({"metric": "FP64 CG solve latency, 4^3 affine hexahedra, N=7, tol 1e-8",
                  "value": p50 * 1e3, "unit": "ms", "higher_is_better": False,
                  "p50_ms": p50 * 1e3, "p99_ms": _pct(times, 99) * 1e3,
                  "iters": res["iters"], "us_per_iter": p50 / res["iters"] * 1e6,
                  "rel_res_true": res_t["rel_res_true"], "max_err_vs_exact_u": err,
                  "oracle_iters": it_o, "rel_diff_vs_oracle_x": xd, "geom": args.geom,
                  "cpu_baseline": {"value": t_cpu * 1e3, "unit": "ms per solve",
                                   "cores": oracle.num_threads(), "kind": "oracle",
                                   "sample": "one full FP64 oracle solve of the same problem"},
                  "dtype": "f64", "data": "synthetic", "config": {"workload": "4^3 N=7 FP64 CG"}})


def run_config3(args):
    """Mixed precision (FP32 inner CG, FP64 outer refinement) against plain
    FP64 CG, both to a true relative residual of 1e-10, 24^3 deformed
    hexahedra, N = 9, manufactured forcing."""
    import torch

    import paper_2108_12188_amd as sem
    from seminputs import MESH_SEED_BASE, box_mesh
    nel = args.nel if args.nel != 32 else 24
    mesh = box_mesh(nel, nel, nel, 9, perturb=0.1, seed=MESH_SEED_BASE + 3)
    gm = sem.Mesh.from_box(mesh, g_fp32=True, g_fp64=True)
    n = mesh.n_local
    xyz = gm.coords()
    b = gm.rhs(_forcing(xyz), prec=sem.FP64)
    u = _exact(xyz)
    out = {}
    for label, prec, geom in (("mixed_otf", sem.MIXED, sem.ON_THE_FLY),
                              ("mixed_pre", sem.MIXED, sem.PRECOMPUTED),
                              ("fp64_pre", sem.FP64, sem.PRECOMPUTED)):
        gm.cg_solve(b, prec=prec, geom=geom, tol=1e-3, max_iter=50)      # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, r = gm.cg_solve(b, prec=prec, geom=geom, tol=1e-10, max_iter=100000,
                           true_residual=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[label] = {"seconds": dt, "iters": r["iters"], "outer": r["outer"],
                      "rel_res_true": r["rel_res_true"], "converged": r["converged"],
                      "gdof_iter_per_s": n * r["iters"] / dt / 1e9,
                      "max_err_vs_exact_u": float((x - u).abs().max())}
        out[label]["x"] = x
    xf = out["fp64_pre"].pop("x")
    for k in ("mixed_otf", "mixed_pre"):
        xm = out[k].pop("x")
        out[k]["rel_diff_vs_fp64_x"] = gm.dot(xm - xf, xm - xf) ** 0.5 / gm.dot(xf, xf) ** 0.5
    best = min(out["mixed_otf"]["seconds"], out["mixed_pre"]["seconds"])
    return _emit({"metric": "time to 1e-10 true residual, 24^3 deformed N=9: mixed vs FP64",
                  "value": best, "unit": "s", "higher_is_better": False,
                  "speedup_vs_fp64": out["fp64_pre"]["seconds"] / best, "runs": out,
                  "n_local": n, "dtype": "f32+f64", "data": "synthetic",
                  "config": {"workload": f"{nel}^3 N=9 +-10% deformed, manufactured, 1e-10"}})


def _batch_problems(count, seed):
    from seminputs import batch_problems, box_mesh
    out = []
    for spec in batch_problems(count, seed=seed):
        out.append(box_mesh(spec["nx"], spec["ny"], spec["nz"], spec["N"], perturb=0.1,
                            seed=spec["seed"]))
    return out


def run_config4(args):
    """64 independent problems (element counts log-uniform 8^3..20^3, N in
    {5, 7, 9}, deformed), mixed precision to 1e-8 in one batch, against the
    same problems solved one after the other (mixed, and plain FP64 to
    1e-10)."""
    import torch

    import paper_2108_12188_amd as sem
    from seminputs import MESH_SEED_BASE
    geom = sem.PRECOMPUTED if args.geom == "pre" else sem.ON_THE_FLY
    boxes = _batch_problems(64, MESH_SEED_BASE + 4)
    meshes = [sem.Mesh.from_box(bx, g_fp32=True, g_fp64=True) for bx in boxes]
    bs = [m.rhs(_forcing(m.coords()), prec=sem.FP64) for m in meshes]
    n_tot = sum(m.n for m in meshes)
    batch = sem.Batch(meshes)
    batch.solve(bs, prec=sem.MIXED, geom=geom, tol=1e-3)       # warm: graphs, workspaces
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, res = batch.solve(bs, prec=sem.MIXED, geom=geom, tol=1e-8)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    work = sum(m.n * r["iters"] for m, r in zip(meshes, res))
    seq_mixed, seq_fp64, lat = 0.0, 0.0, []
    for m, b in zip(meshes, bs):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m.cg_solve(b, prec=sem.MIXED, geom=geom, tol=1e-8)
        torch.cuda.synchronize()
        seq_mixed += time.perf_counter() - t1
        lat.append(time.perf_counter() - t1)
        t1 = time.perf_counter()
        m.cg_solve(b, prec=sem.FP64, geom=sem.PRECOMPUTED, tol=1e-10)
        torch.cuda.synchronize()
        seq_fp64 += time.perf_counter() - t1
    batch.close()
    return _emit({"metric": "batched mixed-precision CG, 64 problems, GDOF*iter/s",
                  "value": work / t_batch / 1e9, "unit": "GDOF·iter/s", "higher_is_better": True,
                  "makespan_s": t_batch, "sequential_mixed_s": seq_mixed,
                  "sequential_fp64_1e-10_s": seq_fp64,
                  "speedup_vs_sequential_mixed": seq_mixed / t_batch,
                  "speedup_vs_sequential_fp64": seq_fp64 / t_batch,
                  "solo_latency_p50_s": _pct(lat, 50), "solo_latency_p99_s": _pct(lat, 99),
                  "all_converged": all(r["converged"] for r in res),
                  "max_rel_res_true": max(r["rel_res_true"] for r in res),
                  "problems": len(meshes), "n_local_total": n_tot, "geom": args.geom,
                  "dtype": "f32+f64", "data": "synthetic",
                  "config": {"workload": "64 problems 8^3..20^3, N in {5,7,9}, mixed to 1e-8"}})


class _Fp64Engine:
    """Plain FP64 CG serving for comparison: the admitted requests are solved
    one at a time, in admission order, each with sem_cg_solve(FP64) to the
    same tolerance (no batching, no mixed precision).  Same interface as
    serve.GpuEngine."""

    def __init__(self, make_problem, tol, geom, prep_workers=4):
        import concurrent.futures as cf

        import torch

        import paper_2108_12188_amd as sem
        self.sem, self.torch = sem, torch
        self.make_problem, self.tol, self.geom = make_problem, tol, geom
        self.pool = cf.ThreadPoolExecutor(max_workers=prep_workers)
        self.preparing, self.order = {}, []
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def wait_until(self, t):
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)

    def footprint(self, r):
        n = r.n_elem * (r.order + 1) ** 3
        return self.sem.mesh_footprint(r.n_elem, r.order, g_fp32=False, g_fp64=True,
                                       prec=self.sem.FP64) + 64 * n

    def _prepare(self, r):
        sem = self.sem
        vert, gid, dirichlet, N, forcing = self.make_problem(r)
        mesh = sem.Mesh(vert, gid, dirichlet, N, g_fp32=False,
                        g_fp64=self.geom == sem.PRECOMPUTED)
        b = mesh.rhs(forcing(mesh.coords()).contiguous(), prec=sem.FP64)
        self.torch.cuda.current_stream().synchronize()
        return mesh, b

    def admit(self, r):
        self.preparing[r.tag] = self.pool.submit(self._prepare, r)
        self.order.append(r.tag)

    def step(self):
        if not self.order:
            return []
        tag = self.order.pop(0)
        mesh, b = self.preparing.pop(tag).result()
        _, res = mesh.cg_solve(b, prec=self.sem.FP64, geom=self.geom, tol=self.tol,
                               max_iter=100000, true_residual=True)
        mesh.close()
        return [(tag, res)]

    def release(self, tag):
        pass

    def close(self):
        self.pool.shutdown(wait=True)


def run_config5(args):
    """Serving: seeded Poisson arrivals of solve requests (4^3..24^3 deformed
    hexahedra, N in {5, 7, 9}, mixed precision to 1e-8); continuous batching
    with admission by device-memory footprint; latency p50/p99 and solves/s.

    The arrival rate defaults to 0.8 x the measured batched capacity: the
    first 256 requests of the stream, prepared in advance and solved as four
    batches of 64 (mixed, to 1e-8), give solves/s.  The same stream is then served
    at that rate and at 0.5 x the capacity, and once more at 0.8 x by plain
    FP64 CG (one solve at a time, same tolerance) for comparison."""
    import torch

    import paper_2108_12188_amd as sem
    from paper_2108_12188_amd.serve import GpuEngine, Request, Scheduler, summarize
    from seminputs import MESH_SEED_BASE, arrival_times, batch_problems, box_mesh
    geom = sem.PRECOMPUTED if args.geom == "pre" else sem.ON_THE_FLY
    specs = batch_problems(args.requests, seed=MESH_SEED_BASE + 5, e_lo=4 ** 3, e_hi=24 ** 3)

    def make_problem(r):
        sp = r.payload
        bx = box_mesh(sp["nx"], sp["ny"], sp["nz"], sp["N"], perturb=0.1, seed=sp["seed"])
        return bx.vert, bx.glob_id, bx.dirichlet, sp["N"], _forcing

    # batched capacity on a sample of the stream (skipped with --no-extras
    # when the rate is given): its first 256 requests
    # (their mean work is within 3% of the whole stream's; the first 64
    # alone carry only three quarters of it), solved as four batches of 64
    import concurrent.futures as cf
    k = min(256, len(specs))
    skip_capacity = args.no_extras and args.rate > 0
    if not skip_capacity:
        log(f"bench5: capacity from the first {k} requests in batches of 64")

    def prep(sp):
        bx = box_mesh(sp["nx"], sp["ny"], sp["nz"], sp["N"], perturb=0.1, seed=sp["seed"])
        m = sem.Mesh.from_box(bx, g_fp32=geom == sem.PRECOMPUTED)
        b = m.rhs(_forcing(m.coords()), prec=sem.FP64)
        torch.cuda.current_stream().synchronize()
        return m, b

    t_cap, all_conv = 0.0, True
    with cf.ThreadPoolExecutor(max_workers=8) as pool:
        for c0 in (range(0, k, 64) if not skip_capacity else ()):
            prepared = list(pool.map(prep, specs[c0:min(k, c0 + 64)]))
            meshes = [m for m, _ in prepared]
            bs = [b for _, b in prepared]
            batch = sem.Batch(meshes)
            if c0 == 0:
                batch.solve(bs, prec=sem.MIXED, geom=geom, tol=1e-3)       # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, bres = batch.solve(bs, prec=sem.MIXED, geom=geom, tol=1e-8)
            torch.cuda.synchronize()
            t_cap += time.perf_counter() - t0
            all_conv &= all(r["converged"] for r in bres)
            batch.close()
            for m in meshes:
                m.close()
            del prepared, meshes, bs
    capacity = k / t_cap if t_cap > 0 else None
    if capacity:
        log(f"bench5: batched capacity {capacity:.1f} solves/s")

    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    rate_main = args.rate if args.rate > 0 else 0.8 * capacity
    runs = {}

    def serve(label, rate, fp64=False):
        arr = arrival_times(len(specs), rate, seed=MESH_SEED_BASE + 50)
        reqs = [Request(tag=q, arrival=float(arr[q]), n_elem=sp["nx"] * sp["ny"] * sp["nz"],
                        order=sp["N"], payload=sp) for q, sp in enumerate(specs)]
        log(f"bench5: {label}: {len(reqs)} requests at {rate:.1f}/s")
        if fp64:
            eng = _Fp64Engine(make_problem, 1e-8, geom, prep_workers=8)
        else:
            eng = GpuEngine(make_problem, tol=1e-8, geom=geom, round_iters=args.round_iters,
                            prep_workers=8)
        t_run = time.perf_counter()

        def progress(k):
            if k % 100 == 0:
                log(f"bench5: {label}: {k} done after {time.perf_counter() - t_run:.1f} s")

        sch = Scheduler(eng, budget_bytes=budget, max_slots=args.slots, on_done=progress)
        out = sch.run(reqs)
        eng.close()
        st = summarize(out)
        st.update({"arrival_rate_per_s": rate, "peak_admitted_bytes": sch.peak_used,
                   "max_rel_res_true": max((r.result or {}).get("rel_res_true", 0.0)
                                           for r in out),
                   "not_converged": [r.tag for r in out if r.status != "done"]})
        if not fp64:
            st["peak_measured_bytes"] = eng.peak_measured_bytes
            st["host_time_s"] = dict(eng.timing)
        log(f"bench5: {label}: p50 {st['p50_s']:.3f} s, p99 {st['p99_s']:.3f} s, "
            f"{st['solves_per_s']:.1f} solves/s")
        runs[label] = st
        return st

    main_run = serve("mixed_0.8x" if args.rate <= 0 else "mixed", rate_main)
    if args.rate <= 0:
        serve("mixed_0.5x", 0.5 * capacity)
    if not args.no_extras:
        serve("fp64_0.8x" if args.rate <= 0 else "fp64", rate_main, fp64=True)
    return _emit({"metric": "serving: solve latency p50 (arrival to result)",
                  "value": main_run["p50_s"], "unit": "s", "higher_is_better": False,
                  "p50_s": main_run["p50_s"], "p99_s": main_run["p99_s"],
                  "solves_per_s": main_run["solves_per_s"],
                  "batched_capacity_solves_per_s": capacity,
                  "capacity_sample": f"first {k} requests solved as batches of 64 (mixed, "
                                     f"1e-8), {t_cap:.2f} s, all converged: {all_conv}",
                  "arrival_rate_per_s": rate_main, "runs": runs,
                  "budget_bytes": budget, "geom": args.geom, "dtype": "f32+f64",
                  "data": "synthetic",
                  "config": {"workload": f"{len(specs)} requests, 4^3..24^3, N in {{5,7,9}}, "
                                         f"mixed to 1e-8, Poisson arrivals at "
                                         f"{rate_main:.1f}/s (plain FP64 CG serving of the same "
                                         f"stream for comparison)"}})


def run_config6(args):
    """Jacobi-preconditioned CG against plain CG.  (a) Cost of one
    iteration: FP32, on-the-fly G, 500 fixed iterations on the 32^3 N=7
    mesh of the headline line, per-kernel times, and the roofline of the
    preconditioned update (it also reads M^-1 and writes z).  (b) Time to a
    true relative residual of 1e-10 (mixed precision, on-the-fly G) with and
    without Jacobi on the 24^3 N=9 deformed mesh (manufactured forcing) and
    on a 24^3 N=7 mesh graded along z (elements ten times thinner at one
    face; random continuous RHS).  (c) The oracle's PCG on this host's
    cores, on a bounded sample of (a)."""
    import numpy as np
    import torch

    import oracle
    import paper_2108_12188_amd as sem
    from seminputs import MESH_SEED_BASE, RHS_SEED, box_mesh, graded_z, random_global_rhs
    nel, N, iters = args.nel, args.order, args.iters
    out = {}
    # (a) iteration cost at the headline size
    log(f"bench6: {nel}^3 N={N} iteration cost")
    mesh = box_mesh(nel, nel, nel, N, perturb=0.1, seed=MESH_SEED_BASE + 2)
    b_host = random_global_rhs(mesh, seed=RHS_SEED)
    n = mesh.n_local
    gm = sem.Mesh.from_box(mesh, g_fp32=True, g_fp64=False)
    b = torch.as_tensor(b_host.astype(np.float32), device="cuda")
    x = torch.zeros_like(b)
    cost = {}
    for label, pc in (("cg", sem.PRECOND_NONE), ("pcg", sem.PRECOND_JACOBI)):
        x.zero_()
        gm.cg_solve(b, x=x, prec=sem.FP32, geom=sem.ON_THE_FLY, fixed_iters=20, precond=pc)
        torch.cuda.synchronize()
        reps = max(1, args.steps)
        t0 = time.perf_counter()
        for _ in range(reps):
            x.zero_()
            gm.cg_solve(b, x=x, prec=sem.FP32, geom=sem.ON_THE_FLY, fixed_iters=iters,
                        precond=pc)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        x.zero_()
        _, prof = gm.cg_solve(b, x=x, prec=sem.FP32, geom=sem.ON_THE_FLY, fixed_iters=iters,
                              precond=pc, kernel_times=True)
        cost[label] = {"gdof_iter_per_s": n * iters / dt / 1e9, "ms_per_iter": 1e3 * dt / iters,
                       "kernel_ms": prof["kernel_ms"]}
    info = gm.info()
    shared_frac = info["n_shared"] / n
    upd_ms = cost["pcg"]["kernel_ms"]["update"]
    table_free = bool(info["gs_table_free"])
    upd_gbs = update_bytes_per_point(N, shared_frac, jacobi=True, table_free=table_free) * n \
        / (upd_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": upd_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": upd_gbs / HBM_PEAK_GBS, "traffic": None,
            "kernel": "%s<float, PC> (gather + mask + r update + z = M^-1 r + <r,z,c>, "
                      "<r,r,c> partials) and the one-block rho finalize, timed together "
                      "between HIP events" % ("update_struct_kernel" if table_free
                                              else "update_gather_kernel"),
            "avg_ms": upd_ms}
    out["iteration_cost"] = cost
    # (c) oracle PCG on a bounded sample of the same mesh
    cpu = None
    if not args.no_cpu:
        log("bench6: oracle PCG CPU baseline")
        pr = oracle.Problem(mesh)
        minv = pr.jacobi_minv()
        k = 2
        t0 = time.perf_counter()
        pr.pcg(b_host, minv=minv, fixed=k)
        t = time.perf_counter() - t0
        if t < 5.0:
            k = max(k, min(200, int(k * 15.0 / max(t, 1e-3))))
            t0 = time.perf_counter()
            pr.pcg(b_host, minv=minv, fixed=k)
            t = time.perf_counter() - t0
        cpu = {"value": n * k / t / 1e9, "unit": "GDOF·iter/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{k} FP64 Jacobi-PCG iterations of the oracle on the {nel}^3 N={N} "
                         f"mesh (diagonal setup excluded); {t:.1f} s timed"}
        del pr
    gm.close()
    del b, x
    # (b) time to 1e-10
    solves = {}
    cases = (("deformed_24_N9", box_mesh(24, 24, 24, 9, perturb=0.1, seed=MESH_SEED_BASE + 3),
              "manufactured"),
             ("graded_24_N7", graded_z(box_mesh(24, 24, 24, 7, perturb=0.1,
                                                seed=MESH_SEED_BASE + 6), s=3.0), "random"))
    for name, m, rhs in cases:
        log(f"bench6: time to 1e-10 on {name}")
        g = sem.Mesh.from_box(m, g_fp32=True, g_fp64=False)
        if rhs == "manufactured":
            bb = g.rhs(_forcing(g.coords()), prec=sem.FP64)
        else:
            bb = torch.as_tensor(random_global_rhs(m, seed=RHS_SEED + 6), device="cuda")
        row = {}
        for label, pc in (("cg", sem.PRECOND_NONE), ("pcg", sem.PRECOND_JACOBI)):
            g.cg_solve(bb, prec=sem.MIXED, geom=sem.ON_THE_FLY, tol=1e-3, max_iter=50,
                       precond=pc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, r = g.cg_solve(bb, prec=sem.MIXED, geom=sem.ON_THE_FLY, tol=1e-10,
                              max_iter=100000, precond=pc)
            torch.cuda.synchronize()
            row[label] = {"seconds": time.perf_counter() - t0, "iters": r["iters"],
                          "outer": r["outer"], "rel_res_true": r["rel_res_true"],
                          "converged": r["converged"]}
        row["speedup"] = row["cg"]["seconds"] / row["pcg"]["seconds"]
        row["n_local"] = m.n_local
        solves[name] = row
        g.close()
    out["time_to_1e10"] = solves
    value = solves["graded_24_N7"]["pcg"]["seconds"]
    return _emit({"metric": "time to 1e-10 true residual with Jacobi-PCG (mixed, on-the-fly G), "
                            "24^3 N=7 graded mesh",
                  "value": value, "unit": "s", "higher_is_better": False,
                  "speedup_vs_cg": solves["graded_24_N7"]["speedup"], "runs": out,
                  "dtype": "f32+f64", "data": "synthetic",
                  "config": {"workload": "Jacobi-PCG vs CG: iteration cost on 32^3 N=7, time to "
                                         "1e-10 on 24^3 N=9 deformed and 24^3 N=7 graded"},
                  "roofline": roof, "cpu_baseline": cpu})


def run_config7(args):
    """FP32 CG throughput against the element count (the analogue of the
    paper's plots over mesh sizes, Sec. 7): near-cubic boxes of 2^7 ... 2^15
    hexahedra (4x4x8 up to 32^3), N = 7, deformed by +-10%, a random
    continuous RHS, 500 fixed iterations, on-the-fly and precomputed G; the
    median of 3 solves after a warm-up."""
    import numpy as np
    import torch

    import paper_2108_12188_amd as sem
    from seminputs import MESH_SEED_BASE, RHS_SEED, box_mesh, random_global_rhs
    N, iters = args.order, args.iters
    points = []
    for ex in range(7, 16):
        a = ex // 3
        b_ = (ex - a) // 2
        dims = (1 << a, 1 << b_, 1 << (ex - a - b_))
        mesh = box_mesh(*dims, N, perturb=0.1, seed=MESH_SEED_BASE + 2)
        n = mesh.n_local
        gm = sem.Mesh.from_box(mesh, g_fp32=True, g_fp64=False)
        b = torch.as_tensor(random_global_rhs(mesh, seed=RHS_SEED).astype(np.float32),
                            device="cuda")
        x = torch.zeros_like(b)
        row = {"elements": 1 << ex, "dims": list(dims), "n_local": n}
        for gname, geom in (("otf", sem.ON_THE_FLY), ("pre", sem.PRECOMPUTED)):
            gm.cg_solve(b, x=x, prec=sem.FP32, geom=geom, fixed_iters=50)
            ts = []
            for _ in range(3):
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                gm.cg_solve(b, x=x, prec=sem.FP32, geom=geom, fixed_iters=iters)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            t = sorted(ts)[1]
            row[f"{gname}_gdof_iter_per_s"] = n * iters / t / 1e9
            row[f"{gname}_us_per_iter"] = t / iters * 1e6
        log(f"bench7: E={1 << ex} {dims}: otf {row['otf_gdof_iter_per_s']:.1f} "
            f"({row['otf_us_per_iter']:.1f} us/iter), pre {row['pre_gdof_iter_per_s']:.1f} "
            f"GDOF*iter/s")
        points.append(row)
        gm.close()
        del b, x
    top = points[-1]
    return _emit({"metric": "FP32 CG GDOF·iter/s against the element count, N=7, 500 iterations",
                  "value": top["otf_gdof_iter_per_s"], "unit": "GDOF·iter/s",
                  "higher_is_better": True, "n_gpus": 1, "points": points,
                  "dtype": "f32", "data": "synthetic",
                  "config": {"workload": "near-cubic boxes of 128 ... 32768 hexahedra, N=7, "
                                         "+-10% deformed, random continuous RHS"}})


def unstructured_rows(args, orders=("structured", "shuffled", "hilbert", "morton", "rows"),
                      steps: int = 3):
    """FP32 CG throughput of the headline workload on the same 32^3 N = 7
    deformed box stored as an unstructured mesh would hold it: elements in a
    seeded random order with each local frame rotated by one of the 24 cube
    rotations ("shuffled"), then that mesh renumbered along a Hilbert or
    Morton curve through the element centroids, or in rows of the centroids
    quantized to the element size (sem_element_order), beside
    the lexicographic box ("structured").  Same geometry and right-hand side
    in every case (only the numbering differs)."""
    import dataclasses

    import numpy as np
    import torch

    import paper_2108_12188_amd as sem
    from seminputs import MESH_SEED_BASE, RHS_SEED, box_mesh, random_global_rhs
    nel, N, iters = args.nel, args.order, args.iters
    geom = sem.PRECOMPUTED if args.geom == "pre" else sem.ON_THE_FLY
    rows = {}
    for label in orders:
        shuffled = label != "structured"
        mesh = box_mesh(nel, nel, nel, N, perturb=0.1, seed=MESH_SEED_BASE + 2,
                        permute=shuffled, reorient=shuffled)
        bh = random_global_rhs(mesh, seed=RHS_SEED)
        if label in ("hilbert", "morton", "rows"):
            kind = {"hilbert": sem.ORDER_HILBERT, "morton": sem.ORDER_MORTON,
                    "rows": sem.ORDER_ROWS}[label]
            t0 = time.perf_counter()
            perm = sem.element_order(mesh.vert, kind)
            t_order = time.perf_counter() - t0
            v, gid, d, bh = sem.permute_elements(perm, mesh.vert, mesh.glob_id, mesh.dirichlet,
                                                 bh)
            mesh = dataclasses.replace(mesh, vert=v, glob_id=gid, dirichlet=d)
        gm = sem.Mesh.from_box(mesh, g_fp32=geom == sem.PRECOMPUTED)
        b = torch.as_tensor(bh.astype(np.float32), device="cuda")
        x = torch.zeros_like(b)
        gm.cg_solve(b, x=x, prec=sem.FP32, geom=geom, fixed_iters=50)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            _, r = gm.cg_solve(b, x=x, prec=sem.FP32, geom=geom, fixed_iters=iters)
            if r["iters"] != iters or r["status"] != 2:
                raise RuntimeError(f"a timed solve stopped early: {r}")
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        x.zero_()
        _, prof = gm.cg_solve(b, x=x, prec=sem.FP32, geom=geom, fixed_iters=iters,
                              kernel_times=True)
        info = gm.info()
        rows[label] = {"gdof_iter_per_s": mesh.n_local * iters / dt / 1e9,
                       "ms_per_solve": dt * 1e3, "kernel_ms": prof["kernel_ms"],
                       "rel_res_recursive": r["rel_res_recursive"],
                       "gather_form": "table-free" if info["gs_table_free"] else "per-point table"}
        if label in ("hilbert", "morton", "rows"):
            rows[label]["order_seconds_host"] = t_order
        log(f"bench: {label}: {rows[label]['gdof_iter_per_s']:.1f} GDOF*iter/s "
            f"{prof['kernel_ms']}")
        gm.close()
        del b, x
    base = rows.get("structured", {}).get("gdof_iter_per_s")
    if base:
        for label, row in rows.items():
            row["vs_structured"] = row["gdof_iter_per_s"] / base
    return rows


def run_config8(args):
    """The headline FP32 CG on unstructured element numberings, with and
    without reordering (see unstructured_rows)."""
    rows = unstructured_rows(args)
    # the value: the best of the three reorderings of the shuffled mesh
    best = max(("hilbert", "morton", "rows"), key=lambda k: rows[k]["gdof_iter_per_s"])
    return _emit({"metric": "FP32 CG GDOF·iter/s, 32^3 N=7: shuffled and rotated elements, "
                            "Hilbert / Morton / row reordered (value: the best), structured",
                  "value": rows[best]["gdof_iter_per_s"], "best_reorder": best,
                  "unit": "GDOF·iter/s",
                  "higher_is_better": True, "rows": rows, "dtype": "f32", "data": "synthetic",
                  "config": {"workload": "32^3 N=7 +-10% deformed, 500 FP32 CG iterations, "
                                         "element numbering varied"}})


def run_config9(args):
    """The paper's performance model (Sec. 5.2, Eq. 15; Table 2) on MI355X.

    For the three solver versions of Table 2 (FP32 with G rematerialized on
    the fly, FP32 with precomputed G, FP64 with precomputed G) on the
    headline 32^3 N = 7 mesh, two schedules of the same CG iteration:
    * "pass": the paper's, the gather-scatter QQ^T a pass of its own over w
      (mesh flag SEM_MESH_GATHER_PASS);
    * "fused": this library's, the face sums gathered inside the update and
      only the edge and vertex groups summed by a small kernel.
    Per-kernel times come from HIP events around every launch of 200
    iterations; the iteration time from solves replayed from graphs.
    Observed beta_gs = the gather-scatter words / the gather-scatter
    kernel's time (the paper's 2 n_gs for the pass schedule, n_gs the shared
    local points, exact); observed beta_eff = the algorithmic words of every
    other kernel / their time.  Model
    parameters measured on kernels that do nothing else: beta_eff = a
    1 GiB device copy, beta_gs = a random-permutation gather and scatter of
    4-byte values over the same vector length (fully unaligned accesses,
    the paper's reference case).  Eq. 15,
    T_c = (Q - Q_gs) / beta_eff + Q_gs / beta_gs, then gives the iteration
    time of each schedule from the model parameters, and the fused
    schedule's from the bandwidths observed on the pass schedule; each is
    compared with the measured time.  Words are 4 bytes (FP32 versions) or
    8 bytes (FP64); cycles are 2.4 GHz engine cycles."""
    import numpy as np
    import torch

    import paper_2108_12188_amd as sem
    from seminputs import MESH_SEED_BASE, RHS_SEED, box_mesh, random_global_rhs
    nel, N = args.nel, args.order
    iters = min(args.iters, 200)
    mesh = box_mesh(nel, nel, nel, N, perturb=0.1, seed=MESH_SEED_BASE + 2)
    n = mesh.n_local
    E = mesh.E
    P3 = (N + 1) ** 3
    bh = random_global_rhs(mesh, seed=RHS_SEED)

    # model parameters from kernels that do nothing else
    def timed(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return sorted(a.elapsed_time(b) for a, b in ev)[reps // 2] * 1e-3

    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").uniform_()
    dst = torch.empty_like(src)
    t_copy = timed(lambda: dst.copy_(src))
    copy_bps = 2 * src.numel() * 4 / t_copy
    # one-direction context for the kernels' fractions of the 8 TB/s peak:
    # torch's sum of the 1 GiB vector (reads) and torch's fill (writes); the
    # sum is torch's reduction, not a read-ceiling measurement
    acc = torch.empty((), dtype=torch.float32, device="cuda")
    read_bps = src.numel() * 4 / timed(lambda: torch.sum(src, 0, out=acc))
    write_bps = dst.numel() * 4 / timed(lambda: dst.fill_(1.0))
    del src, dst, acc
    g = torch.Generator(device="cpu").manual_seed(RHS_SEED)
    perm = torch.randperm(n, generator=g).to("cuda")
    v = torch.rand(n, device="cuda")
    out = torch.empty_like(v)
    t_gather = timed(lambda: torch.index_select(v, 0, perm, out=out))
    t_scatter = timed(lambda: out.index_copy_(0, perm, v))
    # words moved at random per index: one load (gather) or one store
    # (scatter); the index stream itself is sequential
    rand_wps = 2 * n / (t_gather + t_scatter)
    del perm, v, out

    def wpc(bytes_per_s, word):
        return bytes_per_s / word / CLOCK_HZ

    versions = (("FP32-CG-Remat.", sem.FP32, sem.ON_THE_FLY, 4),
                ("FP32-CG", sem.FP32, sem.PRECOMPUTED, 4),
                ("FP64-CG", sem.FP64, sem.PRECOMPUTED, 8))
    edge_slots = 12 * N - 4

    def stream_bytes(sched, geom, word, n_gs):
        """Algorithmic bytes per iteration of everything but the
        gather-scatter: the CG-fused operator (r and p_old read, p written,
        x read and written, w written; precomputed G 6 words per point, or
        the 8 vertices, 24 words, per element), its compact copy of the edge nodes in
        the fused schedule, and the update (r read and written, w read; the
        pass schedule's plain update also reads a code byte per point, the
        fused one the element records and the gathered face values)."""
        op = 6 * word * n + (6 * word * n if geom == sem.PRECOMPUTED else 24 * word * E)
        if sched == "pass":
            return op + (3 * word + 1) * n
        op += word * E * edge_slots
        rec = 8 * (6 + edge_slots) * E
        return op + 3 * word * n + rec + word * n_gs

    rows = {}
    for sched in ("pass", "fused"):
        gm = sem.Mesh.from_box(mesh, g_fp32=True, g_fp64=True, gather_pass=(sched == "pass"))
        info = gm.info()
        n_gs = info["n_shared"]
        for name, prec, geom, word in versions:
            dt = torch.float32 if prec == sem.FP32 else torch.float64
            b = torch.as_tensor(bh, dtype=dt, device="cuda")
            x = torch.zeros_like(b)
            gm.cg_solve(b, x=x, prec=prec, geom=geom, fixed_iters=20)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                x.zero_()
                gm.cg_solve(b, x=x, prec=prec, geom=geom, fixed_iters=iters)
            torch.cuda.synchronize()
            t_iter = (time.perf_counter() - t0) / (2 * iters)
            x.zero_()
            _, pr = gm.cg_solve(b, x=x, prec=prec, geom=geom, fixed_iters=iters,
                                kernel_times=True)
            km = pr["kernel_ms"]
            sb = stream_bytes(sched, geom, word, n_gs)
            # gather-scatter words: the paper's 2 n_gs for the pass; the
            # fused schedule sums only the edge and vertex groups, from the
            # compact copy (each copy read once, one sum per group written;
            # counted as two words per edge slot, an upper bound)
            gs_words = 2 * n_gs if sched == "pass" else 2 * E * edge_slots
            t_gs = km["gs"] * 1e-3
            t_rest = (km["ax"] + km["update"]) * 1e-3
            row = {"n": n, "n_gs": n_gs, "stream_words": sb / word, "gs_words": gs_words,
                   "iteration_us": t_iter * 1e6, "kernel_us": {k: v * 1e3 for k, v in km.items()},
                   "beta_eff_obs": sb / word / t_rest / CLOCK_HZ,
                   "beta_gs_obs": gs_words / t_gs / CLOCK_HZ,
                   "beta_eff_model": wpc(copy_bps, word),
                   "beta_gs_model": rand_wps / CLOCK_HZ,
                   "gs_share_of_iteration": t_gs / t_iter,
                   "gdof_iter_per_s": n / t_iter / 1e9}
            # Eq. 15 with the model parameters
            row["T_c_model_us"] = 1e6 * (sb / word / (row["beta_eff_model"] * CLOCK_HZ) +
                                         gs_words / (row["beta_gs_model"] * CLOCK_HZ))
            row["model_over_measured"] = row["T_c_model_us"] / row["iteration_us"]
            if sched == "fused":
                # Eq. 15 with the bandwidths observed on the pass schedule:
                # a prediction of this schedule from the paper's one
                ps = rows[name]["pass"]
                tc = sb / word / (ps["beta_eff_obs"] * CLOCK_HZ) + \
                    gs_words / (ps["beta_gs_obs"] * CLOCK_HZ)
                row["T_c_from_pass_betas_us"] = tc * 1e6
                row["from_pass_over_measured"] = tc * 1e6 / row["iteration_us"]
            rows.setdefault(name, {})[sched] = row
            log(f"bench9: {sched} {name}: {t_iter * 1e6:.1f} us/iter, beta_eff "
                f"{row['beta_eff_obs']:.1f}, beta_gs {row['beta_gs_obs']:.1f} words/cycle")
            del b, x
        gm.close()
    return _emit({"metric": "Eq. 15 performance model on MI355X (Table 2 analogue): observed "
                            "and modelled beta_eff, beta_gs in words/cycle, 32^3 N=7",
                  "value": rows["FP32-CG-Remat."]["pass"]["beta_gs_obs"],
                  "unit": "words/cycle (beta_gs, FP32 remat, pass schedule)",
                  "higher_is_better": True, "rows": rows,
                  "machine": {"clock_hz": CLOCK_HZ, "copy_GBps": copy_bps / 1e9,
                              "torch_sum_read_GBps": read_bps / 1e9,
                              "torch_fill_write_GBps": write_bps / 1e9,
                              "random_gather_scatter_Gwords_per_s": rand_wps / 1e9,
                              "hbm_peak_words_per_cycle_fp32": HBM_PEAK_GBS * 1e9 / 4 / CLOCK_HZ},
                  "dtype": "f32/f64", "data": "synthetic",
                  "config": {"workload": f"{nel}^3 N={N} +-10% deformed, random RHS, {iters} "
                                         f"CG iterations per version and schedule"}})


SUITES = {1: run_config1, 3: run_config3, 4: run_config4, 5: run_config5, 6: run_config6,
          7: run_config7, 8: run_config8, 9: run_config9}


if __name__ == "__main__":
    sys.exit(main())
