"""Independent dense brute force of the SEM Poisson system (NumPy).

Written separately from ``oracle/`` to pin it: nodes from NumPy's Legendre
routines, weights from the moment equations, Lagrange polynomials built
explicitly from their roots, Jacobians from the interpolated node
coordinates, explicit 3x3 inverses, and element matrices assembled into a
dense global matrix with the scatter map (Eq. 4-5 written out as
A^e_ab = sum_q w_q |J_q| (J_q^-T grad phi_a) . (J_q^-T grad phi_b)).
Only for tiny meshes (N <= 4, a handful of elements).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


def gll_nodes(N: int) -> np.ndarray:
    """Endpoints plus the roots of L_N' (NumPy's Legendre-series routines)."""
    c = np.zeros(N + 1)
    c[N] = 1.0
    inner = np.sort(np.real(npleg.legroots(npleg.legder(c)))) if N >= 2 else np.array([])
    return np.concatenate([[-1.0], inner, [1.0]])


def gll_weights_by_moments(xi: np.ndarray) -> np.ndarray:
    """Weights that integrate 1, x, ..., x^N exactly on [-1, 1]."""
    P = xi.size
    V = np.vander(xi, P, increasing=True).T            # V[k][j] = xi_j^k
    mom = np.array([(1.0 - (-1.0) ** (k + 1)) / (k + 1) for k in range(P)])
    return np.linalg.solve(V, mom)


def lagrange_polys(xi: np.ndarray):
    """Power-series coefficients of the Lagrange polynomials through xi."""
    out = []
    for j in range(xi.size):
        others = np.delete(xi, j)
        c = nppoly.polyfromroots(others)
        out.append(c / nppoly.polyval(xi[j], c))
    return out


def lagrange_deriv_matrix(xi: np.ndarray) -> np.ndarray:
    """Dl[i][j] = l_j'(xi_i), by differentiating the explicit polynomials."""
    polys = lagrange_polys(xi)
    return np.array([[nppoly.polyval(x, nppoly.polyder(polys[j])) for j in range(xi.size)]
                     for x in xi])


def trilinear_points(vert_e: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Physical position of every node (i fastest) of one element: [P^3][3]."""
    P = xi.size
    pts = np.zeros((P ** 3, 3))
    for k in range(P):
        for j in range(P):
            for i in range(P):
                s = np.zeros(3)
                for c in range(2):
                    for b in range(2):
                        for a in range(2):
                            wgt = ((1 + (2 * a - 1) * xi[i]) / 2) * ((1 + (2 * b - 1) * xi[j]) / 2) \
                                * ((1 + (2 * c - 1) * xi[k]) / 2)
                            s += wgt * vert_e[a + 2 * b + 4 * c]
                pts[i + P * (j + P * k)] = s
    return pts


def element_matrix(vert_e: np.ndarray, N: int):
    """Dense A^e [P^3][P^3] and mass diagonal B^e for one element."""
    xi = gll_nodes(N)
    w = gll_weights_by_moments(xi)
    Dl = lagrange_deriv_matrix(xi)
    P = N + 1
    X = trilinear_points(vert_e, xi)                   # nodal coordinates
    n = P ** 3
    A = np.zeros((n, n))
    B = np.zeros(n)
    idx = [(i, j, k) for k in range(P) for j in range(P) for i in range(P)]
    for q, (i, j, k) in enumerate(idx):
        # reference gradients of every basis function at node q: [n][3]
        grad = np.zeros((n, 3))
        for a, (ia, ja, ka) in enumerate(idx):
            grad[a, 0] = Dl[i, ia] * (j == ja) * (k == ka)
            grad[a, 1] = (i == ia) * Dl[j, ja] * (k == ka)
            grad[a, 2] = (i == ia) * (j == ja) * Dl[k, ka]
        J = X.T @ grad                                 # J[d][r] = dX_d/dxi_r
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        phys = grad @ Jinv                             # rows: grad_x phi_a = J^-T grad phi_a
        wq = w[i] * w[j] * w[k]
        A += wq * detJ * (phys @ phys.T)
        B[q] = wq * detJ
    return A, B, X


def assemble(vert: np.ndarray, glob_id: np.ndarray, n_glob: int, N: int):
    """Global dense stiffness, lumped mass and nodal coordinates."""
    E = vert.shape[0]
    A = np.zeros((n_glob, n_glob))
    Bg = np.zeros(n_glob)
    Xg = np.zeros((n_glob, 3))
    Xl = []
    Bl = []
    for e in range(E):
        Ae, Be, Xe = element_matrix(vert[e], N)
        g = glob_id[e]
        A[np.ix_(g, g)] += Ae
        np.add.at(Bg, g, Be)
        Xg[g] = Xe
        Xl.append(Xe)
        Bl.append(Be)
    return A, Bg, Xg, np.concatenate(Xl), np.concatenate(Bl)
