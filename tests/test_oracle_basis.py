"""Pins of the oracle's GLL points/weights and derivative matrix (Sec. 3).

Each check uses something other than the oracle's own formulas: closed
forms from tests/golden/, NumPy's Legendre routines, quadrature exactness,
polynomial exactness of D, the summation-by-parts identity and exact 1D
stiffness integrals from Gauss-Legendre quadrature.
"""
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly

import oracle
from dense_reference import gll_nodes, gll_weights_by_moments, lagrange_deriv_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden_gll():
    out = {}
    env = {"sqrt": math.sqrt, "__builtins__": {}}
    with open(os.path.join(GOLDEN, "gll_closed_forms.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, nodes, wts = [s.strip() for s in line.split("|")]
            out[int(n)] = (np.array([eval(t, env) for t in nodes.split(",")]),
                           np.array([eval(t, env) for t in wts.split(",")]))
    return out


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_closed_forms(N):
    xi_ref, w_ref = _read_golden_gll()[N]
    xi, w = oracle.gll(N)
    np.testing.assert_allclose(xi, xi_ref, atol=1e-15)
    np.testing.assert_allclose(w, w_ref, rtol=1e-14)


@pytest.mark.parametrize("N", range(2, 16))
def test_gll_against_numpy_legendre(N):
    xi, w = oracle.gll(N)
    np.testing.assert_allclose(xi, gll_nodes(N), atol=1e-13)
    assert abs(w.sum() - 2.0) < 1e-13
    # quadrature is exact for polynomials of degree <= 2N-1
    for k in range(2 * N):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13, (N, k)
    # and not for degree 2N (sanity: catches a Gauss-point mistake)
    exact = 2.0 / (2 * N + 1)
    assert abs(np.dot(w, xi ** (2 * N)) - exact) > 1e-11


@pytest.mark.parametrize("N", range(2, 12))
def test_gll_weights_match_moments(N):
    xi, w = oracle.gll(N)
    np.testing.assert_allclose(w, gll_weights_by_moments(xi), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("N", range(1, 12))
def test_deriv_polynomial_exactness(N):
    xi, _ = oracle.gll(N)
    D = oracle.deriv(N, xi)
    assert np.max(np.abs(D @ np.ones(N + 1))) < 1e-12
    for k in range(1, N + 1):
        err = np.max(np.abs(D @ xi ** k - k * xi ** (k - 1)))
        assert err < 1e-11 * max(1, k * N), (N, k, err)


@pytest.mark.parametrize("N", range(2, 9))
def test_deriv_against_explicit_lagrange(N):
    xi, _ = oracle.gll(N)
    np.testing.assert_allclose(oracle.deriv(N, xi), lagrange_deriv_matrix(xi), atol=1e-9)


@pytest.mark.parametrize("N", range(1, 12))
def test_summation_by_parts(N):
    # W D + (W D)^T = diag(-1, 0, ..., 0, 1): discrete integration by parts
    xi, w = oracle.gll(N)
    WD = np.diag(w) @ oracle.deriv(N, xi)
    Bnd = np.zeros((N + 1, N + 1))
    Bnd[0, 0], Bnd[N, N] = -1.0, 1.0
    np.testing.assert_allclose(WD + WD.T, Bnd, atol=1e-13)


@pytest.mark.parametrize("N", range(2, 10))
def test_1d_stiffness_exact(N):
    # K = D^T W D must equal int l_i' l_j' (integrand degree 2N-2 <= 2N-1)
    xi, w = oracle.gll(N)
    D = oracle.deriv(N, xi)
    K = D.T @ np.diag(w) @ D
    gx, gw = npleg.leggauss(N + 4)
    from dense_reference import lagrange_polys
    dp = [nppoly.polyder(c) for c in lagrange_polys(xi)]
    Kex = np.array([[np.sum(gw * nppoly.polyval(gx, a) * nppoly.polyval(gx, b)) for b in dp]
                    for a in dp])
    np.testing.assert_allclose(K, Kex, atol=1e-10 * N * N)


def test_stiffness_N2_golden():
    rows = []
    with open(os.path.join(GOLDEN, "stiffness_N2.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([float(t) for t in line.split()])
    K_ref = np.array(rows) / 6.0
    xi, w = oracle.gll(2)
    D = oracle.deriv(2, xi)
    np.testing.assert_allclose(D.T @ np.diag(w) @ D, K_ref, atol=1e-15)
