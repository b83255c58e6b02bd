"""Reference-element data: quadrature and Lagrange bases (Section 3.2: P_{r+1}
velocity / porous pressures and P_r conduit pressure, r = 1, i.e. P2 and P1).

Reference triangle: vertices (0,0), (1,0), (0,1); barycentrics
l0 = 1 - xi - eta, l1 = xi, l2 = eta.  P2 node order on an element:
vertices 0, 1, 2, then edge midpoints (0,1), (1,2), (0,2).
"""
import numpy as np
from scipy.special import roots_legendre


def gauss_legendre_01(m):
    """m-point Gauss-Legendre rule on [0, 1] (exact to degree 2m-1)."""
    g, w = roots_legendre(m)
    return (g + 1.0) / 2.0, w / 2.0


def triangle_rule(m):
    """Collapsed (Duffy) tensor Gauss-Legendre rule on the reference triangle.

    (u, v) in [0,1]^2 -> xi = u, eta = v (1 - u), Jacobian (1 - u).  Exact for
    polynomials of total degree <= 2m - 2.  Returns points (n, 2), weights (n,)
    summing to the triangle area 1/2.
    """
    g, w = gauss_legendre_01(m)
    U, V = np.meshgrid(g, g, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    pts = np.stack([U.ravel(), (V * (1.0 - U)).ravel()], axis=1)
    wts = (WU * WV * (1.0 - U)).ravel()
    return pts, wts


def p1_basis(pts):
    """P1 values (n, 3) and reference gradients (3, 2)."""
    xi, eta = pts[:, 0], pts[:, 1]
    val = np.stack([1.0 - xi - eta, xi, eta], axis=1)
    grad = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    return val, grad


def p2_basis(pts):
    """P2 values (n, 6) and reference gradients (n, 6, 2)."""
    lam, dlam = p1_basis(pts)
    l0, l1, l2 = lam[:, 0], lam[:, 1], lam[:, 2]
    val = np.stack([
        l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
        4 * l0 * l1, 4 * l1 * l2, 4 * l0 * l2], axis=1)
    n = pts.shape[0]
    grad = np.zeros((n, 6, 2))
    for i in range(3):
        grad[:, i, :] = (4 * lam[:, i] - 1)[:, None] * dlam[i][None, :]
    for k, (i, j) in enumerate([(0, 1), (1, 2), (0, 2)]):
        grad[:, 3 + k, :] = 4 * (lam[:, i][:, None] * dlam[j][None, :]
                                 + lam[:, j][:, None] * dlam[i][None, :])
    return val, grad


def p2_edge_basis(s):
    """1D P2 basis on an edge parametrised by s in [0,1]: end 0, midpoint, end 1.
    Values (n, 3) and d/ds (n, 3)."""
    val = np.stack([(1 - s) * (1 - 2 * s), 4 * s * (1 - s), s * (2 * s - 1)], axis=1)
    der = np.stack([4 * s - 3, 4 - 8 * s, 4 * s - 1], axis=1)
    return val, der
