"""Reference-element data in 3D (Section 3.2 with d = 3: P2 velocity and porous
pressures, P1 conduit pressure on tetrahedra).

Reference tetrahedron: vertices (0,0,0), (1,0,0), (0,1,0), (0,0,1);
barycentrics l0 = 1 - xi - eta - zeta, l1 = xi, l2 = eta, l3 = zeta.
P2 node order on an element: vertices 0..3, then edge midpoints of the edges
(0,1), (0,2), (0,3), (1,2), (1,3), (2,3).
"""
import numpy as np

from .fe import gauss_legendre_01

EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def tet_rule(m):
    """Collapsed (Duffy) tensor Gauss-Legendre rule on the reference tetrahedron.

    (u, v, w) in [0,1]^3 -> xi = u, eta = v (1 - u), zeta = w (1 - u)(1 - v),
    Jacobian (1 - u)^2 (1 - v).  Exact for polynomials of total degree
    <= 2m - 3.  Returns points (n, 3) and weights (n,) summing to the volume 1/6.
    """
    g, w = gauss_legendre_01(m)
    U, V, Wz = np.meshgrid(g, g, g, indexing="ij")
    WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
    xi = U
    eta = V * (1.0 - U)
    zeta = Wz * (1.0 - U) * (1.0 - V)
    pts = np.stack([xi.ravel(), eta.ravel(), zeta.ravel()], axis=1)
    wts = (WU * WV * WW * (1.0 - U) ** 2 * (1.0 - V)).ravel()
    return pts, wts


def p1_basis3(pts):
    """P1 values (n, 4) and reference gradients (4, 3)."""
    xi, eta, zeta = pts[:, 0], pts[:, 1], pts[:, 2]
    val = np.stack([1.0 - xi - eta - zeta, xi, eta, zeta], axis=1)
    grad = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    return val, grad


def p2_basis3(pts):
    """P2 values (n, 10) and reference gradients (n, 10, 3)."""
    lam, dlam = p1_basis3(pts)
    n = pts.shape[0]
    val = np.zeros((n, 10))
    grad = np.zeros((n, 10, 3))
    for i in range(4):
        val[:, i] = lam[:, i] * (2 * lam[:, i] - 1)
        grad[:, i, :] = (4 * lam[:, i] - 1)[:, None] * dlam[i][None, :]
    for k, (i, j) in enumerate(EDGES):
        val[:, 4 + k] = 4 * lam[:, i] * lam[:, j]
        grad[:, 4 + k, :] = 4 * (lam[:, i][:, None] * dlam[j][None, :] + lam[:, j][:, None] * dlam[i][None, :])
    return val, grad
