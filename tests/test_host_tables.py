"""Host logic of the gather inside the CG update: the library's table builder
(sem_tables.cpp) and the gather functions the update kernel calls, compiled
for the CPU and checked point by point against the copies of every global
id (tests/host/gather_tables_check.cpp).  No GPU is used."""
import os
import subprocess

import numpy as np
import pytest

from seminputs import box_mesh

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("host") / "gather_tables_check")
    cmd = [HIPCC, "-x", "hip", "--cuda-host-only", "-O1", "-std=c++17",
           os.path.join(HERE, "host", "gather_tables_check.cpp"),
           os.path.join(ROOT, "paper_2108_12188_amd", "csrc", "sem_tables.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(checker, tmp_path, mesh, glob_id=None):
    gid = mesh.glob_id if glob_id is None else glob_id
    g, d = str(tmp_path / "gid.bin"), str(tmp_path / "dir.bin")
    np.ascontiguousarray(gid, dtype=np.int64).tofile(g)
    np.ascontiguousarray(mesh.dirichlet, dtype=np.uint8).tofile(d)
    r = subprocess.run([checker, str(mesh.E), str(mesh.N), g, d, "12188"], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return dict(kv.split("=") for kv in r.stdout.split())


@pytest.mark.parametrize("shape,N", [((3, 2, 2), 5), ((4, 3, 2), 7), ((2, 2, 2), 9),
                                     ((5, 4, 3), 3), ((3, 3, 3), 1), ((3, 2, 3), 2),
                                     ((2, 2, 1), 11)])
def test_conforming_meshes_gather_in_update(checker, tmp_path, shape, N):
    mesh = box_mesh(*shape, N, perturb=0.1, seed=40 + N, reorient=True, permute=True)
    out = _run(checker, tmp_path, mesh)
    assert out["gs_in_update"] == "1"
    assert int(out["checked"]) == mesh.E * (N + 1) ** 3
    assert int(out["gs_blocks"]) > 0     # block order checked over every block
    if min(shape) > 1:   # interior edges exist: groups with m > 2 on element edges
        assert out["gsum_wedge"] == "1"
    # odd orders also take the table-free form (P^3 a multiple of 4), checked
    # point by point the same way
    assert out["table_free"] == ("1" if N % 2 else "0")
    assert int(out["checked_tf"]) == (mesh.E * (N + 1) ** 3 if N % 2 else 0)


def test_odd_multiplicities_take_the_generic_loop(checker, tmp_path):
    """Moving one copy of a face node into another face node's group makes a
    group of 3: the group sums cover any m, not only 4 and 8."""
    mesh = box_mesh(3, 2, 2, 4, perturb=0.1, seed=7)
    P = mesh.N + 1
    gid = mesh.glob_id.copy()
    # face-interior node (N, 2, 2) of element 0 is shared with element 1;
    # element 5's copy of its own (0, 2, 2) face node joins that group
    face = mesh.N + P * (2 + P * 2)
    other = 0 + P * (2 + P * 2)
    gid[5, other] = gid[0, face]
    out = _run(checker, tmp_path, mesh, gid)
    assert out["gs_in_update"] == "1"
    assert int(out["odd_m"]) == 3
    assert out["gsum_wedge"] == "0"   # a group of face-interior nodes


def test_face_group_of_three_keeps_the_table(checker, tmp_path):
    """At odd N a face-interior node shared by three copies has no single
    partner: the table-free form declines and the per-point table (still
    checked bitwise) is used."""
    mesh = box_mesh(3, 2, 2, 5, perturb=0.1, seed=8)
    P = mesh.N + 1
    gid = mesh.glob_id.copy()
    face = mesh.N + P * (2 + P * 2)
    other = 0 + P * (2 + P * 2)
    gid[5, other] = gid[0, face]
    out = _run(checker, tmp_path, mesh, gid)
    assert out["gs_in_update"] == "1"
    assert out["table_free"] == "0"
    assert int(out["checked"]) == mesh.E * P ** 3


def test_interior_tie_disables_gather_in_update(checker, tmp_path):
    mesh = box_mesh(3, 2, 2, 4, perturb=0.1, seed=2111)
    P = mesh.N + 1
    centre = 2 + P * (2 + P * 2)
    gid = mesh.glob_id.copy()
    gid[1, centre] = gid[0, centre]
    out = _run(checker, tmp_path, mesh, gid)
    assert out["gs_in_update"] == "0"
