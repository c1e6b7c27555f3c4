"""Element orders for locality on unstructured meshes (sem_element_order,
host only): the result is a permutation; along the Hilbert order every two
consecutive cells of a 2^k grid are face neighbours (the defining property of
the curve); the Morton order equals the sort by interleaved coordinate bits
computed here independently; the row order gives a structured box back in
its row-major numbering, deformed or not, with the axis of most cells
slowest; the order does not depend on the input numbering of the elements;
bad arguments are refused."""
import numpy as np
import pytest

from seminputs import box_mesh


def _cells(mesh, n):
    c = mesh.vert.mean(axis=1)
    return np.rint(c * n - 0.5).astype(np.int64)


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_hilbert_steps_are_face_neighbours(n):
    import paper_2108_12188_amd as sem
    m = box_mesh(n, n, n, 1)
    p = sem.element_order(m.vert, sem.ORDER_HILBERT)
    assert sorted(p.tolist()) == list(range(n ** 3))
    g = _cells(m, n)[p]
    steps = np.abs(np.diff(g, axis=0)).sum(axis=1)
    assert np.all(steps == 1)


def test_morton_is_the_interleaved_bit_sort():
    import paper_2108_12188_amd as sem
    n = 8
    m = box_mesh(n, n, n, 1, permute=True, seed=3)
    p = sem.element_order(m.vert, sem.ORDER_MORTON)
    g = _cells(m, n)

    def key(c):
        k = 0
        for b in range(2, -1, -1):
            for d in range(3):
                k = (k << 1) | ((int(c[d]) >> b) & 1)
        return k

    want = sorted(range(n ** 3), key=lambda e: key(g[e]))
    assert p.tolist() == want


@pytest.mark.parametrize("perturb", [0.0, 0.1])
def test_rows_order_restores_the_row_major_numbering(perturb):
    import paper_2108_12188_amd as sem
    a = box_mesh(6, 5, 4, 2, perturb=perturb, seed=7)
    b = box_mesh(6, 5, 4, 2, perturb=perturb, seed=7, permute=True)
    pb = sem.element_order(b.vert, sem.ORDER_ROWS)
    # box_mesh numbers elements x fastest, then y, then z: the permuted
    # copy reordered in rows is the unpermuted box (the axis with the most
    # cells, x here, is the slowest of the row order, so compare by cells)
    ca = np.rint((a.vert.mean(axis=1) - a.vert.mean(axis=1).min(axis=0)) * np.array([6, 5, 4]))
    cb = np.rint((b.vert.mean(axis=1) - b.vert.mean(axis=1).min(axis=0)) * np.array([6, 5, 4]))
    want = sorted(range(b.E), key=lambda e: (cb[e, 0], cb[e, 1], cb[e, 2]))
    assert pb.tolist() == want
    # on a cube the ties keep z slowest and x fastest: the box's own order
    c = box_mesh(4, 4, 4, 1, perturb=perturb, seed=8)
    d = box_mesh(4, 4, 4, 1, perturb=perturb, seed=8, permute=True)
    pd = sem.element_order(d.vert, sem.ORDER_ROWS)
    np.testing.assert_array_equal(d.vert[pd], c.vert)
    assert len(ca) == a.E


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_order_is_independent_of_input_numbering(kind):
    import paper_2108_12188_amd as sem
    a = box_mesh(6, 5, 4, 2, perturb=0.1, seed=4)
    b = box_mesh(6, 5, 4, 2, perturb=0.1, seed=4, permute=True)
    pa = sem.element_order(a.vert, kind)
    pb = sem.element_order(b.vert, kind)
    np.testing.assert_array_equal(a.vert[pa], b.vert[pb])


def test_permute_elements_moves_element_blocks():
    import paper_2108_12188_amd as sem
    m = box_mesh(3, 2, 2, 3, permute=True, seed=5)
    p = sem.element_order(m.vert)
    v, gid, d, x = sem.permute_elements(p, m.vert, m.glob_id, m.dirichlet,
                                        np.arange(m.n_local, dtype=np.float64))
    P3 = (m.N + 1) ** 3
    for k, e in enumerate(p):
        np.testing.assert_array_equal(v[k], m.vert[e])
        np.testing.assert_array_equal(gid[k], m.glob_id[e])
        np.testing.assert_array_equal(d[k], m.dirichlet[e])
        np.testing.assert_array_equal(x[k * P3:(k + 1) * P3], np.arange(e * P3, (e + 1) * P3))


def test_bad_arguments_are_refused():
    import paper_2108_12188_amd as sem
    m = box_mesh(2, 2, 2, 1)
    with pytest.raises(sem.SemError):
        sem.element_order(m.vert, 7)
    bad = m.vert.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(sem.SemError):
        sem.element_order(bad)
