#!/usr/bin/env python3
"""Write ``bench_references.json``: FP64 oracle results that the benchmark
reports beside the GPU's, for workloads too large to run the oracle inside a
timed benchmark.  Calls only ``oracle/`` and ``seminputs/``.

* ``headline``: the 32^3 N = 7 deformed mesh (mesh seed 2110) with the random
  continuous right-hand side (seed 12188): the oracle's FP64 CG (Algorithm 1)
  for 500 fixed iterations from x0 = 0; its recursive residual sqrt(rho/rho0)
  and its true relative residual ||b - A x||_c / ||b||_c.
* ``mixed_24_N9``: the 24^3 N = 9 deformed mesh (mesh seed 2111) with the
  manufactured right-hand side (f = 3 pi^2 sin sin sin at the oracle's GLL
  coordinates, b = mask(QQ^T B f)): the oracle's FP64 CG to 1e-12, x*; its
  iteration count, ||x*||_c, and x* at 4096 seeded local points.

Run from the repository root:  python tests/golden/make_bench_references.py
(about 10 minutes on 8 host threads; writes the JSON beside this script).
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from seminputs import MESH_SEED_BASE, RHS_SEED, box_mesh, random_global_rhs  # noqa: E402

SAMPLES = 4096
SAMPLE_SEED = 4096


def sample_indices(n: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    return np.sort(rng.choice(n, size=SAMPLES, replace=False))


def headline():
    mesh = box_mesh(32, 32, 32, 7, perturb=0.1, seed=MESH_SEED_BASE + 2)
    b = random_global_rhs(mesh, seed=RHS_SEED)
    pr = oracle.Problem(mesh)
    t0 = time.perf_counter()
    x, it, hist = pr.cg(b, fixed=500)
    dt = time.perf_counter() - t0
    rr = pr.true_rel_residual(b, x)
    return {"mesh": "32^3 N=7 perturb 0.1 seed 2110", "rhs": "random global, seed 12188",
            "iterations": int(it), "rel_res_recursive": math.sqrt(hist["rho"][it] / hist["rho"][0]),
            "rel_res_true": rr, "oracle_seconds": dt, "threads": oracle.num_threads()}


def mixed_24_n9():
    mesh = box_mesh(24, 24, 24, 9, perturb=0.1, seed=MESH_SEED_BASE + 3)
    pr = oracle.Problem(mesh)
    b, u = pr.rhs_manufactured()
    t0 = time.perf_counter()
    x, it, _ = pr.cg(b, tol=1e-12, max_iter=100000, history=False)
    dt = time.perf_counter() - t0
    idx = sample_indices(mesh.n_local)
    return {"mesh": "24^3 N=9 perturb 0.1 seed 2111", "rhs": "manufactured",
            "tol": 1e-12, "iterations": int(it), "rel_res_true": pr.true_rel_residual(b, x),
            "norm_c": math.sqrt(pr.dot(x, x)), "max_err_vs_exact_u": float(np.max(np.abs(x - u))),
            "sample_seed": SAMPLE_SEED, "sample_index": idx.tolist(),
            "sample_x": x[idx].tolist(), "oracle_seconds": dt, "threads": oracle.num_threads()}


def main():
    out = {"note": "written by tests/golden/make_bench_references.py from the FP64 oracle"}
    out["headline"] = headline()
    print("headline", {k: v for k, v in out["headline"].items()}, flush=True)
    out["mixed_24_N9"] = mixed_24_n9()
    print("mixed_24_N9 iterations", out["mixed_24_N9"]["iterations"],
          "rel_res_true", out["mixed_24_N9"]["rel_res_true"], flush=True)
    with open(os.path.join(HERE, "bench_references.json"), "w") as f:
        json.dump(out, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
