"""Build the HIP library libsem.so for gfx950 (in-tree).

Every translation unit is compiled by hipcc for gfx950 only; the local
operator is compiled once per polynomial order (-DSEM_ORDER=N).  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsem.so")
ORDERS = range(1, 12)
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-x", "hip",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
]
SOURCES = ["sem_ax_dispatch.cpp", "sem_basis.cpp", "sem_mesh.cpp", "sem_tables.cpp", "sem_cg.cpp",
           "sem_api.cpp", "sem_order.cpp", "sem_gs.hip", "sem_vec.hip", "sem_geom.hip", "sem_batch.hip"]


def _compile(src: str, obj: str, extra=()):
    cmd = [HIPCC, *CFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, out: str | None = None,
          defines=(), build_dir: str | None = None) -> str:
    """Compile every translation unit and link `out` (default: libsem.so in
    the package).  `defines` are extra -D flags for every unit."""
    bdir = build_dir or BUILD
    lib = out or LIB
    os.makedirs(bdir, exist_ok=True)
    dflags = [f"-D{d}" for d in defines]
    jobs = jobs or min(16, os.cpu_count() or 4)
    tasks = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for N in ORDERS:
            tasks.append(ex.submit(_compile, "sem_ax_order.hip",
                                   os.path.join(bdir, f"ax_order_{N}.o"),
                                   [f"-DSEM_ORDER={N}", *dflags]))
        for src in SOURCES:
            if os.path.exists(os.path.join(CSRC, src)):
                obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
                tasks.append(ex.submit(_compile, src, obj, dflags))
        objs = [t.result() for t in tasks]
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
