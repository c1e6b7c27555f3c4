"""Pins of the oracle's geometry, local operator, gather-scatter and mask
(Sec. 3, Eq. 4-5; Sec. 4.3, Eq. 9) against closed forms, invariants and an
independent dense brute force (tests/dense_reference.py)."""
import numpy as np
import pytest

import oracle
from dense_reference import assemble, lagrange_polys
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly
from seminputs import box_mesh, random_local


def _kron3(a, b, c):
    # operator on [k][j][i] data with i fastest: kron(k-part, j-part, i-part)
    return np.kron(a, np.kron(b, c))


def test_affine_cube_geometry():
    N, n = 5, 4          # h = 1/4 is exact after the FP32 rounding of vertices
    mesh = box_mesh(n, n, n, N)
    xi, w = oracle.gll(N)
    G, B = oracle.geom(mesh.vert, N, xi, w)
    h = 1.0 / n
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    for e in range(mesh.E):
        np.testing.assert_allclose(G[e, 0], W * h / 2, rtol=1e-13)
        np.testing.assert_allclose(G[e, 3], W * h / 2, rtol=1e-13)
        np.testing.assert_allclose(G[e, 5], W * h / 2, rtol=1e-13)
        assert np.max(np.abs(G[e, [1, 2, 4]])) < 1e-15
        np.testing.assert_allclose(B[e], W * h ** 3 / 8, rtol=1e-13)


@pytest.mark.parametrize("N", [2, 3, 6])
def test_volume_of_deformed_box(N):
    mesh = box_mesh(3, 2, 4, N, perturb=0.1, seed=7, reorient=True, permute=True)
    _, B = oracle.geom(mesh.vert, N)
    # a trilinear Jacobian determinant has degree <= 2 per direction: exact
    assert abs(B.sum() - 1.0) < 1e-13


def test_inverted_element_rejected():
    mesh = box_mesh(1, 1, 1, 3)
    vert = mesh.vert.copy()
    vert[0, [0, 1]] = vert[0, [1, 0]]          # mirror: negative Jacobian
    with pytest.raises(ValueError):
        oracle.geom(vert, 3)


def test_affine_element_is_kronecker_form():
    # A_L on a cube of side h equals (h/2)(K(x)M(x)M + M(x)K(x)M + M(x)M(x)K)
    # with K the exact 1D stiffness (Gauss-Legendre) and M = diag(w).
    N = 4
    mesh = box_mesh(2, 2, 2, N)
    pr = oracle.Problem(mesh)
    h = 0.5
    xi, w = pr.xi, pr.w
    gx, gw = npleg.leggauss(N + 4)
    dp = [nppoly.polyder(c) for c in lagrange_polys(xi)]
    K = np.array([[np.sum(gw * nppoly.polyval(gx, a) * nppoly.polyval(gx, b)) for b in dp]
                  for a in dp])
    M = np.diag(w)
    Aref = (h / 2) * (_kron3(M, M, K) + _kron3(M, K, M) + _kron3(K, M, M))
    P3 = (N + 1) ** 3
    u = random_local(mesh.n_local, seed=3)
    got = pr.ax_local(u).reshape(mesh.E, P3)
    for e in range(mesh.E):
        np.testing.assert_allclose(got[e], Aref @ u.reshape(mesh.E, P3)[e], atol=1e-12)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_local_operator_symmetric_psd_constant_null(N):
    mesh = box_mesh(2, 2, 1, N, perturb=0.1, seed=11, reorient=True)
    pr = oracle.Problem(mesh)
    u = random_local(mesh.n_local, seed=1)
    v = random_local(mesh.n_local, seed=2)
    Au, Av = pr.ax_local(u), pr.ax_local(v)
    P3 = (N + 1) ** 3
    for e in range(mesh.E):
        s = slice(e * P3, (e + 1) * P3)
        a, b = np.dot(v[s], Au[s]), np.dot(u[s], Av[s])
        assert abs(a - b) <= 1e-13 * (abs(a) + abs(b) + 1)
        assert np.dot(u[s], Au[s]) > 0
    ones = np.ones(mesh.n_local)
    assert np.max(np.abs(pr.ax_local(ones))) < 1e-12


@pytest.mark.parametrize("N,shape,perturb", [(2, (1, 1, 1), 0.1), (3, (2, 1, 1), 0.1),
                                             (2, (2, 2, 2), 0.1), (4, (2, 1, 2), 0.1),
                                             (3, (2, 2, 2), 0.0)])
def test_matrix_free_equals_dense_assembly(N, shape, perturb):
    mesh = box_mesh(*shape, N, perturb=perturb, seed=5, reorient=True, permute=True)
    pr = oracle.Problem(mesh)
    A, Bg, Xg, Xl, Bl = assemble(mesh.vert, mesh.glob_id, mesh.n_glob, N)
    rng = np.random.default_rng(9)
    ug = rng.uniform(-1, 1, mesh.n_glob)
    uL = ug[mesh.glob_id.ravel()]
    # QQ^T A_L Q u = Q (A u): the plain definition of the matrix-free operator
    got = pr.gs(pr.ax_local(uL))
    ref = (A @ ug)[mesh.glob_id.ravel()]
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.max(np.abs(ref)))
    # the mass matrix and the node coordinates agree too
    np.testing.assert_allclose(pr.B.ravel(), Bl, rtol=1e-12)
    np.testing.assert_allclose(pr.coords().T, Xl, atol=1e-14)


def test_matrix_free_permutation_invariant():
    N = 3
    m1 = box_mesh(2, 2, 2, N, perturb=0.1, seed=4)
    m2 = box_mesh(2, 2, 2, N, perturb=0.1, seed=4, permute=True, reorient=True)
    p1, p2 = oracle.Problem(m1), oracle.Problem(m2)
    rng = np.random.default_rng(1)
    ug = rng.uniform(-1, 1, m1.n_glob)
    w1 = p1.gs(p1.ax_local(ug[m1.glob_id.ravel()]))
    w2 = p2.gs(p2.ax_local(ug[m2.glob_id.ravel()]))
    g1 = np.zeros(m1.n_glob)
    g2 = np.zeros(m2.n_glob)
    g1[m1.glob_id.ravel()] = w1
    g2[m2.glob_id.ravel()] = w2
    np.testing.assert_allclose(g1, g2, atol=1e-12)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_linear_patch_test(N):
    # GLL quadrature integrates grad(linear).grad(phi) |J| exactly on
    # trilinear elements (degree <= 2N-1), so a linear field is in the
    # kernel of the assembled operator at every interior global point.
    mesh = box_mesh(3, 3, 3, N, perturb=0.1, seed=21, reorient=True)
    pr = oracle.Problem(mesh)
    x, y, z = pr.coords()
    u = 0.3 + 1.7 * x - 0.9 * y + 2.3 * z
    w = pr.gs(pr.ax_local(u))
    interior = mesh.dirichlet.ravel() == 0
    assert np.max(np.abs(w[interior])) < 1e-12


def test_gather_scatter_invariants():
    N = 4
    mesh = box_mesh(3, 2, 2, N, perturb=0.1, seed=3, permute=True, reorient=True)
    pr = oracle.Problem(mesh)
    rng = np.random.default_rng(2)
    ug = rng.uniform(-1, 1, mesh.n_glob)
    uL = ug[mesh.glob_id.ravel()]
    # QQ^T (Q u) = m o (Q u)
    np.testing.assert_allclose(pr.gs(uL), pr.m * uL, rtol=1e-15)
    # sum_l c_l (QQ^T v)_l = sum_l v_l (each global sum counted once)
    v = random_local(mesh.n_local, seed=8)
    assert abs(np.sum(pr.gs(v) / pr.m) - np.sum(v)) < 1e-11
    # the weighted inner product of continuous vectors is the global one
    vg = rng.uniform(-1, 1, mesh.n_glob)
    assert abs(pr.dot(uL, vg[mesh.glob_id.ravel()]) - np.dot(ug, vg)) < 1e-12


@pytest.mark.parametrize("n,N", [(4, 7), (3, 5), (2, 9)])
def test_shared_point_counts_against_eq9(n, N):
    # Eq. 9: points on element boundaries, n (P^3 - (N-1)^3) / P^3; the
    # shared local points are those minus the ones on the domain boundary
    # that only one element holds.
    mesh = box_mesh(n, n, n, N)
    pr = oracle.Problem(mesh)
    P = N + 1
    n_gs_eq9 = mesh.n_local * (P ** 3 - (N - 1) ** 3) // P ** 3
    shared = int(np.sum(pr.m > 1))
    assert shared <= n_gs_eq9
    # exact count for a box: every element-boundary point minus those held by
    # one element only (on a cube face but not on an element edge/vertex
    # shared with a neighbour)
    on_elem_bnd = np.zeros(P ** 3, dtype=bool)
    idx = np.arange(P)
    kk, jj, ii = np.meshgrid(idx, idx, idx, indexing="ij")
    on_elem_bnd = ((ii == 0) | (ii == N) | (jj == 0) | (jj == N) | (kk == 0) | (kk == N)).ravel()
    assert np.sum(np.tile(on_elem_bnd, mesh.E)) == n_gs_eq9
    unique_glob = np.unique(mesh.glob_id)
    assert unique_glob.size == (n * N + 1) ** 3
    # multiplicities are 1, 2, 4 or 8 on a box
    assert set(np.unique(pr.m).astype(int)) <= {1, 2, 4, 8}
    assert np.sum(1.0 / pr.m) == pytest.approx((n * N + 1) ** 3)


def test_mask_zeroes_only_boundary():
    mesh = box_mesh(2, 2, 2, 3)
    pr = oracle.Problem(mesh)
    v = random_local(mesh.n_local, seed=1)
    mv = pr.mask(v)
    d = mesh.dirichlet.ravel() != 0
    assert np.all(mv[d] == 0)
    assert np.array_equal(mv[~d], v[~d])
