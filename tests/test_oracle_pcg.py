"""Pins of the oracle's Jacobi-preconditioned CG (the paper's stated future
work: a preconditioner; Jacobi, the diagonal of the assembled operator, is
the first choice).

The diagonal is pinned against the diagonal of the independent dense
assembly (tests/dense_reference.py) and against e_q^T A_L e_q computed with
the oracle's own matrix-free operator on unit vectors.  PCG with the
identity as M^-1 reduces to CG (same histories, bit for bit); with Jacobi it
reaches the dense Cholesky solution; its error in the A-norm decreases
monotonically, as PCG's must; and the one-unknown element converges in one
iteration to pi^2/8, like CG.
"""
import math

import numpy as np
import pytest

import oracle
from dense_reference import assemble
from seminputs import box_mesh, random_global_rhs


@pytest.mark.parametrize("N,shape", [(2, (1, 1, 1)), (3, (2, 1, 1)), (4, (2, 2, 1)),
                                     (3, (2, 2, 2))])
def test_diagonal_equals_dense_assembly(N, shape):
    mesh = box_mesh(*shape, N, perturb=0.12, seed=5, reorient=True, permute=True)
    pr = oracle.Problem(mesh)
    d = pr.diag_A()
    A, *_ = assemble(mesh.vert, mesh.glob_id, mesh.n_glob, N)
    ref = np.diag(A)[mesh.glob_id.ravel()]
    assert np.max(np.abs(d - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_diagonal_equals_operator_on_unit_vectors():
    mesh = box_mesh(2, 1, 2, 3, perturb=0.1, seed=8)
    pr = oracle.Problem(mesh)
    n, P3 = pr.n, (mesh.N + 1) ** 3
    elem = np.zeros(n)
    for l in range(n):
        e = np.zeros(n)
        e[l] = 1.0
        elem[l] = pr.ax_local(e)[l]          # (A_L)_ll, element by element
    ref = pr.gs(elem)                        # summed over the copies
    assert np.max(np.abs(pr.diag_A() - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_identity_preconditioner_reduces_to_cg():
    mesh = box_mesh(3, 2, 2, 4, perturb=0.1, seed=3)
    pr = oracle.Problem(mesh)
    b = random_global_rhs(mesh)
    ident = np.where(pr.dirichlet.astype(bool), 0.0, 1.0)
    xc, itc, hc = pr.cg(b, fixed=25)
    xp, itp, hp = pr.pcg(b, minv=ident, fixed=25)
    assert itc == itp == 25
    for k in ("rho", "alpha", "beta"):
        assert np.array_equal(hc[k], hp[k]), k
    assert np.array_equal(xc, xp)


@pytest.mark.parametrize("N,shape", [(3, (2, 2, 1)), (4, (2, 1, 2))])
def test_pcg_equals_dense_cholesky(N, shape):
    mesh = box_mesh(*shape, N, perturb=0.15, seed=21, reorient=True, permute=True)
    pr = oracle.Problem(mesh)
    b, _ = pr.rhs_manufactured()
    x, it, _ = pr.pcg(b, tol=1e-13, max_iter=2000)
    A, Bg, Xg, Xl, Bl = assemble(mesh.vert, mesh.glob_id, mesh.n_glob, N)
    fg = 3 * math.pi ** 2 * np.prod(np.sin(math.pi * Xg), axis=1)
    free = np.ones(mesh.n_glob, dtype=bool)
    free[mesh.glob_id.ravel()[mesh.dirichlet.ravel() != 0]] = False
    Aff = A[np.ix_(free, free)]
    xf = np.linalg.solve(Aff, (Bg * fg)[free])
    xg = np.zeros(mesh.n_glob)
    xg[free] = xf
    ref = xg[mesh.glob_id.ravel()]
    assert np.max(np.abs(x - ref)) <= 1e-11 * np.max(np.abs(ref))
    assert it <= int(free.sum()) + 5


def test_pcg_error_decreases_in_the_energy_norm():
    mesh = box_mesh(3, 3, 2, 4, perturb=0.15, seed=4)
    pr = oracle.Problem(mesh)
    b = random_global_rhs(mesh)
    xs, _, _ = pr.pcg(b, tol=1e-14, max_iter=5000)
    prev = math.inf
    for k in range(1, 30):
        xk, _, _ = pr.pcg(b, fixed=k)
        e = xk - xs
        en = pr.dot(e, pr.apply_A(e))       # ||e||_A^2 on the assembled system
        assert en <= prev * (1 + 1e-12) + 1e-300
        prev = en


def test_single_element_one_iteration():
    mesh = box_mesh(1, 1, 1, 2)
    pr = oracle.Problem(mesh)
    b, _ = pr.rhs_manufactured()
    x, it, _ = pr.pcg(b, tol=1e-14, max_iter=10)
    centre = 1 + 3 * (1 + 3 * 1)
    assert it == 1
    assert abs(x[centre] - math.pi ** 2 / 8) <= 1e-14


def test_jacobi_needs_fewer_iterations_on_deformed_mesh():
    mesh = box_mesh(4, 3, 3, 5, perturb=0.2, seed=9)
    pr = oracle.Problem(mesh)
    b = random_global_rhs(mesh)
    _, itc, _ = pr.cg(b, tol=1e-8, max_iter=5000)
    _, itp, _ = pr.pcg(b, tol=1e-8, max_iter=5000)
    assert itp < itc
