"""Autotuner of the local operator: contraction engine and tile shape.

For every (order, precision, geometric-factor form) the tuner times the
CG-fused operator kernel -- the kernel of the solver's iteration -- for
every shape the VALU engine accepts (one thread per (i, j) column, at most
512 threads and 64 KiB of LDS) and, where it is built, the matrix-core
engine (one element per workgroup of one or two waves), with HIP events
inside sem_cg_solve, and keeps the fastest.  Results are stored as JSON keyed by
GPU architecture and applied with sem_ax_engine_set / sem_ax_shape_set.

    python -m paper_2108_12188_amd.tune            # tune N = 5, 7, 9 and save
"""
from __future__ import annotations

import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned_shapes.json")
_PREC = {"fp32": 1, "fp64": 0}
_GEOM = {"pre": 0, "otf": 1}


def candidates(N: int, fp64: bool):
    P2, P3 = (N + 1) ** 2, (N + 1) ** 3
    tsz = 8 if fp64 else 4
    staged = not fp64 and P3 % 4 == 0     # FP32 fused tiles also stage r, p, vertices

    def lds(q):
        return 2 * tsz * q * P3 + (8 * q * P3 + 96 * q if staged else 0)

    out = []
    epb = 1
    while ((epb * P2 + 63) // 64) * 64 <= 512 and lds(epb) <= 65536:
        out.append(epb)
        epb += 1
    return out


def tune_one(N: int, prec: str, geom: str, target_points: int = 8_000_000, iters: int = 20):
    """Returns (best candidate, {candidate: mean fused-operator ms}); a
    candidate is "valu:<elements per block>" or "mfma"."""
    import numpy as np
    import torch

    import paper_2108_12188_amd as sem
    from seminputs import box_mesh, random_global_rhs
    P3 = (N + 1) ** 3
    side = max(2, int(round((target_points / P3) ** (1.0 / 3.0))))
    mesh = box_mesh(side, side, side, N, perturb=0.1, seed=7)
    fp64 = prec == "fp64"
    gm = sem.Mesh.from_box(mesh, g_fp32=not fp64, g_fp64=fp64)
    dt = torch.float64 if fp64 else torch.float32
    b = torch.as_tensor(random_global_rhs(mesh).astype(np.float64), dtype=dt, device="cuda")
    times = {}

    def run(key):
        gm.cg_solve(b, prec=_PREC[prec], geom=_GEOM[geom], fixed_iters=3)
        _, r = gm.cg_solve(b, prec=_PREC[prec], geom=_GEOM[geom], fixed_iters=iters,
                           kernel_times=True)
        times[key] = r["kernel_ms"]["ax"]

    sem.ax_engine_set(N, _PREC[prec], _GEOM[geom], sem.ENGINE_VALU)
    for epb in candidates(N, fp64):
        sem.ax_shape_set(N, _PREC[prec], _GEOM[geom], epb)
        run(f"valu:{epb}")
    sem.ax_shape_set(N, _PREC[prec], _GEOM[geom], 0)
    try:
        sem.ax_engine_set(N, _PREC[prec], _GEOM[geom], sem.ENGINE_MFMA)
        run("mfma")
    except sem.SemError:
        pass                                  # not built for this order / precision
    sem.ax_engine_set(N, _PREC[prec], _GEOM[geom], sem.ENGINE_DEFAULT)
    gm.close()
    best = min(times, key=times.get)
    return best, times


def arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def autotune(orders=(5, 7, 9), precs=("fp32",), geoms=("pre", "otf"), path: str = CACHE):
    entries = []
    for N in orders:
        for prec in precs:
            for geom in geoms:
                best, times = tune_one(N, prec, geom)
                engine = "mfma" if best == "mfma" else "valu"
                epb = 1 if best == "mfma" else int(best.split(":")[1])
                entries.append({"N": N, "prec": prec, "geom": geom, "engine": engine,
                                "elems_per_block": epb, "ax_ms": times})
                print(f"tune N={N} {prec} {geom}: best {best} ({times[best] * 1e3:.1f} us)",
                      flush=True)
    data = {"arch": arch(), "entries": entries}
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    return data


def apply(path: str = CACHE) -> int:
    """Applies the cached shapes that match this GPU; returns how many."""
    import paper_2108_12188_amd as sem
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    if data.get("arch") != arch():
        return 0
    for e in data.get("entries", []):
        p, g = _PREC[e["prec"]], _GEOM[e["geom"]]
        engine = e.get("engine")              # absent: keep the built-in engine
        if engine == "mfma":
            sem.ax_engine_set(e["N"], p, g, sem.ENGINE_MFMA)
        else:
            if engine == "valu":
                sem.ax_engine_set(e["N"], p, g, sem.ENGINE_VALU)
            sem.ax_shape_set(e["N"], p, g, e["elems_per_block"])
    return len(data.get("entries", []))


def main(argv=None):
    ap = argparse.ArgumentParser(description="operator engine and tile-shape autotuner")
    ap.add_argument("--orders", default="5,7,9")
    ap.add_argument("--precs", default="fp32")
    ap.add_argument("--out", default=CACHE)
    a = ap.parse_args(argv)
    autotune(tuple(int(x) for x in a.orders.split(",")), tuple(a.precs.split(",")),
             path=a.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
