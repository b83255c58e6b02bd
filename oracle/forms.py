"""The forms of the weak formulation (Section 3.1, Eq. (3.1) and the definitions
of a_F, a_f, a_m, a_{c,eta}, a_{Gamma,eta}, b_{N,eta}, b_eta) assembled with
scipy.sparse over an arbitrary set of elements of one region mesh.

Unscaled building blocks (coefficients are applied by the scheme):
  mass  M[a,b]  = int phi_a phi_b                       (P2 scalar)
  stiff K[a,b]  = int grad phi_a . grad phi_b           (P2 scalar)
  strain S[(a,c),(b,d)] = int 2 D(phi_b e_d) : D(phi_a e_c)
  div   Bq[q,(b,d)] = int psi_q d_d phi_b                (P1 test, P2 vector trial)
  conv  c(w)[(a,c)] = int ((w . grad) w)_c phi_a
        N(w)[(a,c),(b,d)] = int (phi_b d_d w_c + delta_cd (w . grad phi_b)) phi_a
        (the Newton derivative of c, so N(w) w = 2 c(w))
  Gamma (y = 1, horizontal, tangent e_x, n_c = (0,-1)):
        G[a,b]  = int_Gamma phi_a phi_b
        Gx[a,b] = int_Gamma phi_a d_x phi_b
Vector P2 unknowns are component-blocked: index c * n2^2 + node.
"""
import numpy as np
import scipy.sparse as sps

from .fe import triangle_rule, p1_basis, p2_basis, p2_edge_basis, gauss_legendre_01

QUAD_M = 6          # 36-point collapsed rule, exact to degree 10
EDGE_M = 6          # 6-point Gauss rule on edges, exact to degree 11

_PTS, _WTS = triangle_rule(QUAD_M)
_P2V, _P2G = p2_basis(_PTS)
_P1V, _ = p1_basis(_PTS)


def _geom(mesh, t):
    J = mesh.jacobian(t)
    det = abs(np.linalg.det(J))
    invJ = np.linalg.inv(J)
    grad = _P2G @ invJ            # (nq, 6, 2): row-vector gradients g_xi J^-1
    return J, det, grad


def _coo(rows, cols, vals, shape):
    return sps.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=shape).tocsr()


def _split(mesh, E):
    E = np.asarray(E, dtype=np.int64)
    return [(t, E[mesh.el_orient[E] == t]) for t in (0, 1)]


def p2_mass_stiff(mesh, E):
    """Scalar P2 mass and stiffness over elements E (region numbering)."""
    n = mesh.n2 ** 2
    Ms, Ks = [], []
    for t, Et in _split(mesh, E):
        if len(Et) == 0:
            continue
        _, det, g = _geom(mesh, t)
        w = _WTS * det
        Me = np.einsum("q,qa,qb->ab", w, _P2V, _P2V)
        Ke = np.einsum("q,qak,qbk->ab", w, g, g)
        nodes = mesh.el_p2[Et]
        r = np.repeat(nodes[:, :, None], 6, 2)
        c = np.repeat(nodes[:, None, :], 6, 1)
        Ms.append(_coo(r, c, np.broadcast_to(Me, r.shape), (n, n)))
        Ks.append(_coo(r, c, np.broadcast_to(Ke, r.shape), (n, n)))
    return sum(Ms), sum(Ks)


def stokes_blocks(mesh, E):
    """Vector mass (block diagonal), strain S, and divergence Bq over E."""
    n2 = mesh.n2 ** 2
    n1 = mesh.n1 ** 2
    Mv, Sv, Bv = [], [], []
    for t, Et in _split(mesh, E):
        if len(Et) == 0:
            continue
        _, det, g = _geom(mesh, t)
        w = _WTS * det
        Me = np.einsum("q,qa,qb->ab", w, _P2V, _P2V)
        GG = np.einsum("q,qak,qbk->ab", w, g, g)
        # S[(a,c),(b,d)] = delta_cd grad_a.grad_b + d_d phi_a d_c phi_b
        Se = np.zeros((2, 6, 2, 6))
        for c in range(2):
            for d in range(2):
                Se[c, :, d, :] = (GG if c == d else 0.0) + np.einsum("q,qa,qb->ab", w, g[:, :, d], g[:, :, c])
        Be = np.zeros((3, 2, 6))
        for d in range(2):
            Be[:, d, :] = np.einsum("q,qv,qb->vb", w, _P1V, g[:, :, d])
        nodes = mesh.el_p2[Et]
        vn = mesh.el_p1[Et]
        vidx = np.concatenate([nodes, nodes + n2], axis=1)          # (ne, 12) comp-blocked
        Se12 = Se.reshape(12, 12)
        r = np.repeat(vidx[:, :, None], 12, 2)
        c = np.repeat(vidx[:, None, :], 12, 1)
        Sv.append(_coo(r, c, np.broadcast_to(Se12, r.shape), (2 * n2, 2 * n2)))
        Me12 = np.kron(np.eye(2), Me)
        Mv.append(_coo(r, c, np.broadcast_to(Me12, r.shape), (2 * n2, 2 * n2)))
        rb = np.repeat(vn[:, :, None], 12, 2)
        cb = np.repeat(vidx[:, None, :], 3, 1)
        Bv.append(_coo(rb, cb, np.broadcast_to(Be.reshape(3, 12), rb.shape), (n1, 2 * n2)))
    return sum(Mv), sum(Sv), sum(Bv)


def _w_at_qp(mesh, Et, w, g):
    n2 = mesh.n2 ** 2
    nodes = mesh.el_p2[Et]
    we = np.stack([w[nodes], w[nodes + n2]], axis=1)                 # (ne, 2, 6)
    wq = np.einsum("eca,qa->eqc", we, _P2V)                          # (ne, nq, 2)
    gw = np.einsum("eca,qak->eqck", we, g)                           # (ne, nq, c, k) = d_k w_c
    return nodes, wq, gw


def convection(mesh, E, w):
    """c(w) vector and Newton matrix N(w) of b_N(u,u,v) = ((u.grad)u, v)
    (Section 3.1, trilinear form), over elements E."""
    n2 = mesh.n2 ** 2
    vec = np.zeros(2 * n2)
    mats = []
    for t, Et in _split(mesh, E):
        if len(Et) == 0:
            continue
        _, det, g = _geom(mesh, t)
        wts = _WTS * det
        nodes, wq, gw = _w_at_qp(mesh, Et, w, g)
        adv = np.einsum("eqk,eqck->eqc", wq, gw)                     # (w.grad)w
        ce = np.einsum("q,eqc,qa->eca", wts, adv, _P2V)              # (ne, 2, 6)
        vidx = np.concatenate([nodes, nodes + n2], axis=1)
        np.add.at(vec, vidx.ravel(), ce.reshape(len(Et), 12).ravel())
        # N[(a,c),(b,d)] = sum_q wts (phi_b d_d w_c + delta_cd (w.grad phi_b)) phi_a
        Ne = np.einsum("q,qb,eqcd,qa->ecadb", wts, _P2V, gw, _P2V)
        wgrad = np.einsum("eqk,qbk->eqb", wq, g)
        T = np.einsum("q,eqb,qa->eab", wts, wgrad, _P2V)
        for c in range(2):
            Ne[:, c, :, c, :] += T
        Ne = Ne.reshape(len(Et), 12, 12)
        r = np.repeat(vidx[:, :, None], 12, 2)
        cc = np.repeat(vidx[:, None, :], 12, 1)
        mats.append(_coo(r, cc, Ne, (2 * n2, 2 * n2)))
    return vec, sum(mats)


def load_p2(mesh, E, func):
    """int func(x) phi_a over elements E; func maps (n,2) points to (n,)."""
    n = mesh.n2 ** 2
    out = np.zeros(n)
    for t, Et in _split(mesh, E):
        if len(Et) == 0:
            continue
        J, det, _ = _geom(mesh, t)
        ci = mesh.el_cell[Et]
        v0 = np.stack([ci[:, 0] * mesh.h, mesh.y0 + ci[:, 1] * mesh.h], 1)
        X = v0[:, None, :] + np.einsum("kl,ql->qk", J, _PTS)[None]   # (ne, nq, 2)
        f = func(X.reshape(-1, 2)).reshape(len(Et), -1)
        le = np.einsum("q,eq,qa->ea", _WTS * det, f, _P2V)
        np.add.at(out, mesh.el_p2[Et].ravel(), le.ravel())
    return out


def gamma_forms(mesh, x0=0, x1=None):
    """Edge matrices on Gamma edges of cells x0 <= i < x1 of `mesh`:
    G[a,b] = int phi_a phi_b and Gx[a,b] = int phi_a d_x phi_b (region numbering)."""
    n = mesh.n2 ** 2
    nodes, _ = mesh.gamma_edges(x0, x1)
    s, ws = gauss_legendre_01(EDGE_M)
    val, der = p2_edge_basis(s)
    h = mesh.h
    Ge = h * np.einsum("q,qa,qb->ab", ws, val, val)
    Gxe = np.einsum("q,qa,qb->ab", ws, val, der)       # dx = h ds, d_x = d_s / h
    r = np.repeat(nodes[:, :, None], 3, 2)
    c = np.repeat(nodes[:, None, :], 3, 1)
    G = _coo(r, c, np.broadcast_to(Ge, r.shape), (n, n))
    Gx = _coo(r, c, np.broadcast_to(Gxe, r.shape), (n, n))
    return G, Gx


def gamma_transfer(mesh_from, mesh_to):
    """Map Gamma node values from one region's P2 lattice to the other's (same N):
    sparse (n_to, n_from) selecting node (a, Gamma row)."""
    assert mesh_from.N == mesh_to.N
    a = np.arange(mesh_from.n2)
    bf = 2 * mesh_from.N if mesh_from.region == 0 else 0
    bt = 2 * mesh_to.N if mesh_to.region == 0 else 0
    rows = a + mesh_to.n2 * bt
    cols = a + mesh_from.n2 * bf
    return sps.coo_matrix((np.ones(len(a)), (rows, cols)),
                          shape=(mesh_to.n2 ** 2, mesh_from.n2 ** 2)).tocsr()


def p1_mass(mesh, E):
    """Scalar P1 mass matrix over elements E."""
    n = mesh.n1 ** 2
    Ms = []
    for t, Et in _split(mesh, E):
        if len(Et) == 0:
            continue
        _, det, _ = _geom(mesh, t)
        Me = np.einsum("q,qa,qb->ab", _WTS * det, _P1V, _P1V)
        nodes = mesh.el_p1[Et]
        r = np.repeat(nodes[:, :, None], 3, 2)
        c = np.repeat(nodes[:, None, :], 3, 1)
        Ms.append(_coo(r, c, np.broadcast_to(Me, r.shape), (n, n)))
    return sum(Ms)
