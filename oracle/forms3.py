"""The forms of the weak formulation in 3D (Section 3.1 with d = 3) assembled
with scipy.sparse over an arbitrary set of tetrahedra of one region mesh.

Unscaled building blocks (coefficients are applied by the scheme):
  mass  M[a,b]  = int phi_a phi_b                       (P2 scalar)
  stiff K[a,b]  = int grad phi_a . grad phi_b           (P2 scalar)
  strain S[(a,c),(b,d)] = int 2 D(phi_b e_d) : D(phi_a e_c)
                        = int delta_cd grad phi_a . grad phi_b + d_c phi_b d_d phi_a
  div   Bq[q,(b,d)] = int psi_q d_d phi_b                (P1 test, P2 vector trial)
  conv  c(w)[(a,c)] = int ((w . grad) w)_c phi_a
        N(w)[(a,c),(b,d)] = int (phi_b d_d w_c + delta_cd (w . grad phi_b)) phi_a
        (the Newton derivative of c, so N(w) w = 2 c(w))
  Gamma (z = 1, horizontal, tangents e_x, e_y, n_c = (0,0,-1)):
        G[a,b]   = int_Gamma phi_a phi_b
        Gx[a,b]  = int_Gamma phi_a d_x phi_b,  Gy[a,b] = int_Gamma phi_a d_y phi_b
Vector P2 unknowns are component-blocked: index c * n2^3 + node.
"""
import numpy as np
import scipy.sparse as sps

from .fe import triangle_rule, p2_basis
from .fe3 import tet_rule, p1_basis3, p2_basis3
from .mesh3 import POROUS

QUAD_M = 5          # 125-point collapsed rule, exact to degree 7
LOAD_M = 6          # 216 points, exact to degree 9 (sources)
FACE_M = 6          # 36-point face rule, exact to degree 10

_PTS, _WTS = tet_rule(QUAD_M)
_P2V, _P2G = p2_basis3(_PTS)
_P1V, _ = p1_basis3(_PTS)
_PP = np.einsum("qa,qb->qab", _P2V, _P2V).reshape(len(_WTS), 100)   # phi_a phi_b at the points


def _geom(mesh, r, grads):
    J = mesh.jacobian(r)
    det = abs(np.linalg.det(J))
    invJ = np.linalg.inv(J)
    return det, grads @ invJ          # (nq, nb, 3) physical gradients


def _coo(rows, cols, vals, shape):
    return sps.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=shape).tocsr()


def _split(mesh, E):
    E = np.asarray(E, dtype=np.int64)
    return [(r, E[mesh.el_orient[E] == r]) for r in range(6)]


def p2_mass_stiff(mesh, E):
    """Scalar P2 mass and stiffness over tetrahedra E (region numbering)."""
    n = mesh.n2 ** 3
    Ms, Ks = [], []
    for r, Er in _split(mesh, E):
        if len(Er) == 0:
            continue
        det, g = _geom(mesh, r, _P2G)
        w = _WTS * det
        Me = np.einsum("q,qa,qb->ab", w, _P2V, _P2V)
        Ke = np.einsum("q,qak,qbk->ab", w, g, g)
        nodes = mesh.el_p2[Er]
        rr = np.repeat(nodes[:, :, None], 10, 2)
        cc = np.repeat(nodes[:, None, :], 10, 1)
        Ms.append(_coo(rr, cc, np.broadcast_to(Me, rr.shape), (n, n)))
        Ks.append(_coo(rr, cc, np.broadcast_to(Ke, rr.shape), (n, n)))
    return sum(Ms), sum(Ks)


def stokes_blocks(mesh, E):
    """Vector mass Mv, strain S (3 n2^3 square) and divergence Bq (n1^3 x 3 n2^3)."""
    n2, n1 = mesh.n2 ** 3, mesh.n1 ** 3
    Mv, S, B = [], [], []
    for r, Er in _split(mesh, E):
        if len(Er) == 0:
            continue
        det, g = _geom(mesh, r, _P2G)
        w = _WTS * det
        Me = np.einsum("q,qa,qb->ab", w, _P2V, _P2V)
        Ke = np.einsum("q,qak,qbk->ab", w, g, g)
        nodes = mesh.el_p2[Er]
        pn = mesh.el_p1[Er]
        for c in range(3):
            for d in range(3):
                Se = np.einsum("q,qb,qa->ab", w, g[:, :, c], g[:, :, d])
                if c == d:
                    Se = Se + Ke
                rr = np.repeat(nodes[:, :, None], 10, 2) + c * n2
                cc = np.repeat(nodes[:, None, :], 10, 1) + d * n2
                S.append(_coo(rr, cc, np.broadcast_to(Se, rr.shape), (3 * n2, 3 * n2)))
            rr = np.repeat(nodes[:, :, None], 10, 2) + c * n2
            cc = np.repeat(nodes[:, None, :], 10, 1) + c * n2
            Mv.append(_coo(rr, cc, np.broadcast_to(Me, rr.shape), (3 * n2, 3 * n2)))
            Be = np.einsum("q,qv,qb->vb", w, _P1V, g[:, :, c])
            rr = np.repeat(pn[:, :, None], 10, 2)
            cc = np.repeat(nodes[:, None, :], 4, 1) + c * n2
            B.append(_coo(rr, cc, np.broadcast_to(Be, rr.shape), (n1, 3 * n2)))
    return sum(Mv), sum(S), sum(B)


def convection(mesh, E, w):
    """c(w) (vector of 3 n2^3) and N(w) (3 n2^3 square) over tetrahedra E."""
    n2 = mesh.n2 ** 3
    cv = np.zeros(3 * n2)
    N = []
    for r, Er in _split(mesh, E):
        if len(Er) == 0:
            continue
        det, g = _geom(mesh, r, _P2G)
        wq = _WTS * det
        nodes = mesh.el_p2[Er]
        W = np.stack([w[c * n2 + nodes] for c in range(3)], 1)         # (ne, 3, 10)
        wv = np.einsum("qa,eca->eqc", _P2V, W)                          # w at qp
        gw = np.einsum("qak,eca->eqck", g, W)                           # d_k w_c
        adv = np.einsum("eqk,qbk->eqb", wv, g)                          # w . grad phi_b
        for c in range(3):
            conv_c = np.einsum("eqk,eqk->eq", wv, gw[:, :, c, :])       # (w . grad) w_c
            np.add.at(cv, c * n2 + nodes, (wq * conv_c) @ _P2V)
            for d in range(3):
                # int phi_b d_d w_c phi_a: quadrature weights times the
                # pointwise products phi_a phi_b
                Ne = ((wq * gw[:, :, c, d]) @ _PP).reshape(-1, 10, 10)
                if c == d:
                    Ne = Ne + np.einsum("q,eqb,qa->eab", wq, adv, _P2V, optimize=True)
                rr = np.repeat(nodes[:, :, None], 10, 2) + c * n2
                cc = np.repeat(nodes[:, None, :], 10, 1) + d * n2
                N.append(_coo(rr, cc, Ne, (3 * n2, 3 * n2)))
    return cv, sum(N)


def load_p2(mesh, E, func):
    """int func phi_a over tetrahedra E; func(X (n,3)) -> (n,)."""
    pts, wts = tet_rule(LOAD_M)
    val, _ = p2_basis3(pts)
    n = mesh.n2 ** 3
    out = np.zeros(n)
    c = mesh.p1_coords()
    for r, Er in _split(mesh, E):
        if len(Er) == 0:
            continue
        J = mesh.jacobian(r)
        det = abs(np.linalg.det(J))
        v0 = c[mesh.el_p1[Er, 0]]                                       # (ne, 3)
        X = v0[:, None, :] + np.einsum("ij,qj->qi", J, pts)[None, :, :]  # (ne, nq, 3)
        f = func(X.reshape(-1, 3)).reshape(len(Er), -1)
        np.add.at(out, mesh.el_p2[Er], np.einsum("q,eq,qa->ea", wts * det, f, val))
    return out


def gamma_forms(mesh, x0=0, x1=None, y0=0, y1=None):
    """G, Gx, Gy over the interface triangles of the cells x0 <= i < x1,
    y0 <= j < y1 (n2^3 square, region numbering)."""
    pts, wts = triangle_rule(FACE_M)
    val, grad = p2_basis(pts)
    n = mesh.n2 ** 3
    nodes, ors, _ = mesh.gamma_faces(x0, x1, y0, y1)
    h = mesh.h
    G, Gx, Gy = [], [], []
    for o in (0, 1):
        sel = ors == o
        if not sel.any():
            continue
        # the face triangle's affine map in (x, y), as the 2D mesh's orientation o
        Jf = h * (np.array([[1.0, 1.0], [0.0, 1.0]]) if o == 0 else np.array([[1.0, 0.0], [1.0, 1.0]]))
        det = abs(np.linalg.det(Jf))
        gphys = grad @ np.linalg.inv(Jf)
        w = wts * det
        Ge = np.einsum("q,qa,qb->ab", w, val, val)
        Gxe = np.einsum("q,qa,qb->ab", w, val, gphys[:, :, 0])
        Gye = np.einsum("q,qa,qb->ab", w, val, gphys[:, :, 1])
        nd = nodes[sel]
        rr = np.repeat(nd[:, :, None], 6, 2)
        cc = np.repeat(nd[:, None, :], 6, 1)
        G.append(_coo(rr, cc, np.broadcast_to(Ge, rr.shape), (n, n)))
        Gx.append(_coo(rr, cc, np.broadcast_to(Gxe, rr.shape), (n, n)))
        Gy.append(_coo(rr, cc, np.broadcast_to(Gye, rr.shape), (n, n)))
    return sum(G), sum(Gx), sum(Gy)


def gamma_transfer(mesh_from, mesh_to):
    """Sparse map of Gamma node values from one region's lattice to the other's
    (same (a, b) on Gamma; other entries zero)."""
    L = mesh_from.n2
    a = np.arange(L)
    A, B = np.meshgrid(a, a, indexing="xy")
    A, B = A.ravel(), B.ravel()
    cf = 2 * mesh_from.N if mesh_from.region == POROUS else 0
    ct = 2 * mesh_to.N if mesh_to.region == POROUS else 0
    src = A + L * (B + L * cf)
    dst = A + L * (B + L * ct)
    n = L ** 3
    return sps.coo_matrix((np.ones(len(src)), (dst, src)), shape=(n, n)).tocsr()



def p1_mass(mesh, E):
    """P1 mass over tetrahedra E (pressure norms)."""
    n = mesh.n1 ** 3
    Ms = []
    for r, Er in _split(mesh, E):
        if len(Er) == 0:
            continue
        det = abs(np.linalg.det(mesh.jacobian(r)))
        Me = np.einsum("q,qa,qb->ab", _WTS * det, _P1V, _P1V)
        pn = mesh.el_p1[Er]
        rr = np.repeat(pn[:, :, None], 4, 2)
        cc = np.repeat(pn[:, None, :], 4, 1)
        Ms.append(_coo(rr, cc, np.broadcast_to(Me, rr.shape), (n, n)))
    return sum(Ms)
