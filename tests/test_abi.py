"""CPU checks of the C-ABI library: it is built, loads, and exports every
function that include/sem.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sem.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sem_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("sem_mesh_create", "sem_ax", "sem_gs", "sem_cg_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2108_12188_amd as sem
    path = sem.library_path()
    assert os.path.exists(path), "libsem.so must be built (python paper_2108_12188_amd/build.py)"
    L = ctypes.CDLL(path)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(sem.EXPORTS) == _declared_functions()


def test_version_and_error_string_without_gpu():
    import paper_2108_12188_amd as sem
    assert "gfx950" in sem.version()
    # a message only after a failing call on this thread
    assert isinstance(sem.lib().sem_last_error(), bytes)
    perm = (ctypes.c_int64 * 1)()
    assert sem.lib().sem_element_order(0, None, 0, perm) == -1
    assert b"n_elem" in sem.lib().sem_last_error()


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import paper_2108_12188_amd as sem
    from seminputs import box_mesh
    m = box_mesh(1, 1, 1, 2)
    with pytest.raises(RuntimeError):
        sem.Mesh.from_box(m)
