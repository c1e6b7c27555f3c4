"""Autotuner of the local-operator tile shape (elements per workgroup).

For every (order, precision, geometric-factor form) the tuner times the
CG-fused operator kernel -- the kernel of the solver's iteration -- for
every shape the kernel accepts (one thread per (i, j) column, at most 512
threads and 64 KiB of LDS), with HIP events inside sem_cg_solve, and keeps
the fastest.  Results are stored as JSON keyed by GPU architecture and
applied with sem_ax_shape_set.

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
    """Returns (best epb, {epb: mean fused-operator ms})."""
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
    for epb in candidates(N, fp64):
        sem.ax_shape_set(N, _PREC[prec], _GEOM[geom], epb)
        gm.cg_solve(b, prec=_PREC[prec], geom=_GEOM[geom], fixed_iters=3)
        _, r = gm.cg_solve(b, prec=_PREC[prec], geom=_GEOM[geom], fixed_iters=iters,
                           kernel_times=True)
        times[epb] = r["kernel_ms"]["ax"]
    sem.ax_shape_set(N, _PREC[prec], _GEOM[geom], 0)
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
                entries.append({"N": N, "prec": prec, "geom": geom, "elems_per_block": best,
                                "ax_ms": {str(k): v for k, v in times.items()}})
                print(f"tune N={N} {prec} {geom}: best {best} "
                      f"({times[best] * 1e3:.1f} us; default {times.get(_default(N, prec), 0) * 1e3:.1f} us)",
                      flush=True)
    data = {"arch": arch(), "entries": entries}
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    return data


def _default(N: int, prec: str) -> int:
    import paper_2108_12188_amd as sem
    return sem.ax_shape_get(N, _PREC[prec], 0)["elems_per_block"]


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
        sem.ax_shape_set(e["N"], _PREC[e["prec"]], _GEOM[e["geom"]], e["elems_per_block"])
    return len(data.get("entries", []))


def main(argv=None):
    ap = argparse.ArgumentParser(description="tile-shape autotuner")
    ap.add_argument("--orders", default="5,7,9")
    ap.add_argument("--precs", default="fp32")
    ap.add_argument("--out", default=CACHE)
    a = ap.parse_args(argv)
    autotune(tuple(int(x) for x in a.orders.split(",")), tuple(a.precs.split(",")),
             path=a.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
