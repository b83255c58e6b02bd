"""The discretisation the paper's printed numbers come from (Section 6, first
paragraph): MINI elements in the conduit -- continuous P1 velocity enriched by
one cubic bubble per triangle (P1b), continuous P1 pressure -- and P1 elements
for the three porous pressures, with Algorithm 1 (Section 3.3, partitioned
time stepping) on one grid.  Test infrastructure only, like the rest of this
package.

The same weak form as ``scheme`` (Section 3.1, Eq. (3.1)) with the P2 spaces
replaced; the bubbles are kept as unknowns (no static condensation), so every
matrix is the plain Galerkin matrix of the MINI space.

Unknowns
  porous pressures: P1 vertex values, index i + (N+1) j (the ``mesh`` P1 lattice)
  conduit velocity, per component: the N+1 x N+1 vertex values, then one
      bubble coefficient per element (element id order); component-blocked,
      c * nb + k with nb = (N+1)^2 + 2 N^2
  conduit pressure: P1 vertex values
Bubble: b = 27 l0 l1 l2 (value 1 at the centroid, zero on every edge).

Readings
  M1  initial data (R7 for this element): vertex values of the exact field,
      and the bubble coefficient that makes the element's value at its
      centroid exact (b(centroid) = 1, the P1 part there is the vertex mean).
  M2  Dirichlet data at the boundary vertices; bubbles are interior unknowns.
  M3  Gamma terms act on traces, where the bubbles vanish: the P1 edge forms.
  M5  Algorithm 3: the MINI spaces of T_H and T_h are not nested (a coarse
      bubble is not a fine MINI function), so Pi_h is the fine MINI
      interpolant of the coarse function (its values at the fine vertices,
      bubbles exact at the fine centroids, as M1); the P1 parts are nested
      and prolonged exactly.  The local spaces are the fine functions
      supported in Omega_j: vertices off the artificial faces (velocity and
      pressure, as R1 and R1p) and the bubbles of the elements inside.  The
      merge weights vertices as R4 and takes a bubble from the core holding
      its element.
  M6  the lagged e^n of Eqs. (5.5)-(5.8): the subdomain's own e_j^n, as the
      equations write it ("own", the default and the library's reading), or
      the merged correction of Step 4 restricted to Omega_j and zero on its
      artificial faces ("merged"), offered to compare with Table 1.
"""
import numpy as np
import scipy.sparse as sps

from .fe import triangle_rule, p1_basis, gauss_legendre_01
from .mesh import RegionMesh, POROUS, CONDUIT, make_subdomains, owner_counts
from .mms import MMS
from .scheme import Coefs, _solve_dirichlet, _locate

_PTS, _WTS = triangle_rule(6)              # exact to degree 10
_P1V, _P1G = p1_basis(_PTS)                # (nq, 3), (3, 2)


def mini_basis(pts):
    """Values (n, 4) and reference gradients (n, 4, 2) of the three P1 hats and
    the bubble 27 l0 l1 l2 on the reference triangle."""
    lam, dlam = p1_basis(pts)
    n = pts.shape[0]
    val = np.concatenate([lam, (27.0 * lam[:, 0] * lam[:, 1] * lam[:, 2])[:, None]], axis=1)
    grad = np.zeros((n, 4, 2))
    grad[:, :3, :] = dlam[None]
    l0, l1, l2 = lam[:, 0], lam[:, 1], lam[:, 2]
    grad[:, 3, :] = 27.0 * ((l1 * l2)[:, None] * dlam[0] + (l0 * l2)[:, None] * dlam[1]
                            + (l0 * l1)[:, None] * dlam[2])
    return val, grad


_MBV, _MBG = mini_basis(_PTS)


def n_vel(mesh):
    """Velocity unknowns per component: vertices, then one bubble per element."""
    return mesh.n1 ** 2 + 2 * mesh.N ** 2


def el_vel(mesh, E):
    """(ne, 4) velocity unknowns of elements E: three vertices, then the bubble."""
    E = np.asarray(E, dtype=np.int64)
    return np.concatenate([mesh.el_p1[E], (mesh.n1 ** 2 + E)[:, None]], axis=1)


def _coo(rows, cols, vals, shape):
    return sps.coo_matrix((np.asarray(vals).ravel(), (rows.ravel(), cols.ravel())), shape=shape).tocsr()


def _pairs(idx):
    k = idx.shape[1]
    return np.repeat(idx[:, :, None], k, 2), np.repeat(idx[:, None, :], k, 1)


def _orient(mesh, E):
    E = np.asarray(E, dtype=np.int64)
    for o in (0, 1):
        Et = E[mesh.el_orient[E] == o]
        if len(Et):
            J = mesh.jacobian(o)
            yield o, Et, J, abs(np.linalg.det(J)), np.linalg.inv(J)


def _qp_coords(mesh, Et, J):
    ci = mesh.el_cell[Et]
    v0 = np.stack([ci[:, 0] * mesh.h, mesh.y0 + ci[:, 1] * mesh.h], 1)
    return v0[:, None, :] + np.einsum("kl,ql->qk", J, _PTS)[None]      # (ne, nq, 2)


# ---------------------------------------------------------------------------
# forms of Section 3.1 on the P1 / MINI spaces
# ---------------------------------------------------------------------------
def p1_mass_stiff(mesh, E):
    """Scalar P1 mass and stiffness (porous forms a_F, a_f, a_m and the
    exchange terms) over elements E."""
    n = mesh.n1 ** 2
    M = K = 0
    for _, Et, _, det, invJ in _orient(mesh, E):
        g = _P1G @ invJ                                                # (3, 2)
        Me = np.einsum("q,qa,qb->ab", _WTS * det, _P1V, _P1V)
        Ke = det * _WTS.sum() * (g @ g.T)
        r, c = _pairs(mesh.el_p1[Et])
        M = M + _coo(r, c, np.broadcast_to(Me, r.shape), (n, n))
        K = K + _coo(r, c, np.broadcast_to(Ke, r.shape), (n, n))
    return M, K


def mini_stokes(mesh, E):
    """Vector mass, strain form S[(a,c),(b,d)] = int 2 D(phi_b e_d) : D(phi_a e_c)
    and divergence Bq[q,(b,d)] = int psi_q d_d phi_b (P1 test), MINI trial."""
    nb, n1 = n_vel(mesh), mesh.n1 ** 2
    Mv = Sv = Bv = 0
    for _, Et, _, det, invJ in _orient(mesh, E):
        w = _WTS * det
        g = _MBG @ invJ                                                # (nq, 4, 2)
        Me = np.einsum("q,qa,qb->ab", w, _MBV, _MBV)
        GG = np.einsum("q,qak,qbk->ab", w, g, g)
        Se = np.zeros((2, 4, 2, 4))
        for c in range(2):
            for d in range(2):
                Se[c, :, d, :] = (GG if c == d else 0.0) + np.einsum("q,qa,qb->ab", w, g[:, :, d], g[:, :, c])
        Be = np.stack([np.einsum("q,qv,qb->vb", w, _P1V, g[:, :, d]) for d in range(2)], axis=1)   # (3,2,4)
        vl = el_vel(mesh, Et)
        vidx = np.concatenate([vl, vl + nb], axis=1)                   # (ne, 8)
        r, c = _pairs(vidx)
        Sv = Sv + _coo(r, c, np.broadcast_to(Se.reshape(8, 8), r.shape), (2 * nb, 2 * nb))
        Mv = Mv + _coo(r, c, np.broadcast_to(np.kron(np.eye(2), Me), r.shape), (2 * nb, 2 * nb))
        pn = mesh.el_p1[Et]
        rb = np.repeat(pn[:, :, None], 8, 2)
        cb = np.repeat(vidx[:, None, :], 3, 1)
        Bv = Bv + _coo(rb, cb, np.broadcast_to(Be.reshape(3, 8), rb.shape), (n1, 2 * nb))
    return Mv, Sv, Bv


def mini_convection(mesh, E, w):
    """c(w) = ((w.grad) w, v) and its Newton derivative N(w) (the trilinear form
    of Section 3.1) on the MINI space; N(w) w = 2 c(w)."""
    nb = n_vel(mesh)
    vec = np.zeros(2 * nb)
    mats = 0
    for _, Et, _, det, invJ in _orient(mesh, E):
        wts = _WTS * det
        g = _MBG @ invJ
        vl = el_vel(mesh, Et)
        we = np.stack([w[vl], w[vl + nb]], axis=1)                     # (ne, 2, 4)
        wq = np.einsum("eca,qa->eqc", we, _MBV)
        gw = np.einsum("eca,qak->eqck", we, g)
        adv = np.einsum("eqk,eqck->eqc", wq, gw)
        ce = np.einsum("q,eqc,qa->eca", wts, adv, _MBV)
        vidx = np.concatenate([vl, vl + nb], axis=1)
        np.add.at(vec, vidx.ravel(), ce.reshape(len(Et), 8).ravel())
        Ne = np.einsum("q,qb,eqcd,qa->ecadb", wts, _MBV, gw, _MBV)
        T = np.einsum("q,eqb,qa->eab", wts, np.einsum("eqk,qbk->eqb", wq, g), _MBV)
        for c in range(2):
            Ne[:, c, :, c, :] += T
        r, c = _pairs(vidx)
        mats = mats + _coo(r, c, Ne.reshape(len(Et), 8, 8), (2 * nb, 2 * nb))
    return vec, mats


def load(mesh, E, func, space):
    """int func(x) phi_a over elements E for the P1 ("p1") or MINI ("mini") basis."""
    V, n = (_P1V, mesh.n1 ** 2) if space == "p1" else (_MBV, n_vel(mesh))
    out = np.zeros(n)
    for _, Et, J, det, _ in _orient(mesh, E):
        X = _qp_coords(mesh, Et, J)
        f = func(X.reshape(-1, 2)).reshape(len(Et), -1)
        le = np.einsum("q,eq,qa->ea", _WTS * det, f, V)
        dofs = mesh.el_p1[Et] if space == "p1" else el_vel(mesh, Et)
        np.add.at(out, dofs.ravel(), le.ravel())
    return out


def gamma_p1(mesh, x0=0, x1=None):
    """P1 edge forms on the Gamma edges (y = 1) of cells x0 <= i < x1:
    G[a,b] = int phi_a phi_b and Gx[a,b] = int phi_a d_x phi_b, on the
    region's P1 lattice."""
    n, N, h = mesh.n1 ** 2, mesh.N, mesh.h
    j = N if mesh.region == POROUS else 0
    i = np.arange(x0, N if x1 is None else x1)
    nodes = np.stack([i + mesh.n1 * j, i + 1 + mesh.n1 * j], 1)
    s, ws = gauss_legendre_01(4)
    val = np.stack([1 - s, s], 1)
    der = np.array([-1.0, 1.0])                       # d/ds; d_x = d_s / h, dx = h ds
    Ge = h * np.einsum("q,qa,qb->ab", ws, val, val)
    Gxe = np.einsum("q,qa,b->ab", ws, val, der)
    r, c = _pairs(nodes)
    return (_coo(r, c, np.broadcast_to(Ge, r.shape), (n, n)),
            _coo(r, c, np.broadcast_to(Gxe, r.shape), (n, n)))


def gamma_transfer_p1(mesh_from, mesh_to):
    """Select the Gamma vertices of one region's P1 lattice into the other's."""
    a = np.arange(mesh_from.n1)
    jf = mesh_from.N if mesh_from.region == POROUS else 0
    jt = mesh_to.N if mesh_to.region == POROUS else 0
    return sps.coo_matrix((np.ones(len(a)), (a + mesh_to.n1 * jt, a + mesh_from.n1 * jf)),
                          shape=(mesh_to.n1 ** 2, mesh_from.n1 ** 2)).tocsr()


def dirichlet_p1(mesh):
    """Physical-boundary vertices of a region, Gamma excluded."""
    c = np.arange(mesh.n1 ** 2)
    a, b = c % mesh.n1, c // mesh.n1
    d = (a == 0) | (a == mesh.N)
    return d | ((b == 0) if mesh.region == POROUS else (b == mesh.N))


# ---------------------------------------------------------------------------
# interpolation (M1) and Algorithm 1
# ---------------------------------------------------------------------------
def interp_p1(mesh, mms, name, tt):
    return mms(name, mesh.p1_coords(), tt)


def interp_mini(mesh, mms, name, tt):
    """Vertex values, then per element the bubble coefficient that makes the
    value at the centroid exact."""
    vert = mms(name, mesh.p1_coords(), tt)
    E = np.arange(2 * mesh.N ** 2)
    X = mesh.p1_coords()[mesh.el_p1[E]].mean(axis=1)                # centroids
    bub = mms(name, X, tt) - vert[mesh.el_p1[E]].mean(axis=1)
    return np.concatenate([vert, bub])


class MiniProblem:
    """Constant operators of one grid of N cells per unit length."""

    def __init__(self, N, co, outflow_top=False):
        self.outflow_top = outflow_top
        self.mp = RegionMesh(N, POROUS)
        self.mc = RegionMesh(N, CONDUIT)
        self.co = co
        E = np.arange(2 * N * N)
        self.M, self.K = p1_mass_stiff(self.mp, E)
        self.Mv, self.S, self.Bq = mini_stokes(self.mc, E)
        self.Gp, _ = gamma_p1(self.mp)
        self.Gc, self.Gxc = gamma_p1(self.mc)
        self.T_cp = gamma_transfer_p1(self.mc, self.mp)
        self.T_pc = gamma_transfer_p1(self.mp, self.mc)
        self.dir_p = dirichlet_p1(self.mp)
        nb, n1 = n_vel(self.mc), self.mc.n1 ** 2
        dv = np.zeros(nb, bool)
        dv[:n1] = dirichlet_p1(self.mc)
        if outflow_top:
            # the side walls x = 0, 1 (their end points included) keep u = 0;
            # the rest of the top y = 2 is an outflow boundary (natural)
            i = np.arange(n1) % self.mc.n1
            dv[:n1] = (i == 0) | (i == N)
        self.dir_u = dv


def mini_porous_step(mp_, mms, P_n, U_n, t1):
    """Algorithm 1 Step 1 (the same decoupled SPD systems as Eqs. (5.1)-(5.3)):
    three P1 solves with lagged exchange and the lagged Gamma flux u^n . n_c."""
    co, M, K = mp_.co, mp_.M, mp_.K
    nb = n_vel(mp_.mc)
    n1c = mp_.mc.n1 ** 2
    PF, Pf, Pm = P_n
    E = np.arange(2 * mp_.mp.N ** 2)
    Q = [load(mp_.mp, E, lambda X, nm=nm: mms(nm, X, t1), "p1") for nm in ("qF", "qf", "qm")]
    # u^n . n_c = -u_y on Gamma; only the vertex part of u_y has a trace
    gam = -mp_.Gp @ (mp_.T_cp @ U_n[nb:nb + n1c])
    A = [(co.tau[0] + co.sst) * M + co.kap[0] * K,
         (co.tau[1] + co.s + co.sst) * M + co.kap[1] * K,
         (co.tau[2] + co.s) * M + co.kap[2] * K]
    rhs = [Q[0] + co.tau[0] * (M @ PF) + co.sst * (M @ Pf) + gam,
           Q[1] + co.tau[1] * (M @ Pf) + co.s * (M @ Pm) + co.sst * (M @ PF),
           Q[2] + co.tau[2] * (M @ Pm) + co.s * (M @ Pf)]
    xy = mp_.mp.p1_coords()
    return [_solve_dirichlet(A[i], rhs[i], mp_.dir_p, mms(nm, xy, t1))
            for i, nm in enumerate(("pF", "pf", "pm"))]


def mini_ns_step(mp_, mms, U_n, P_n, PF_n, t1, tol=1e-13, maxit=30, convection=True):
    """Algorithm 1 Step 2: backward Euler Navier-Stokes on the MINI space with
    the lagged p_F on Gamma, solved by Newton's method."""
    co, mc = mp_.co, mp_.mc
    nb, n1 = n_vel(mc), mc.n1 ** 2
    E = np.arange(2 * mc.N ** 2)
    F = np.concatenate([load(mc, E, lambda X: mms("f1", X, t1), "mini"),
                        load(mc, E, lambda X: mms("f2", X, t1), "mini")])
    pg = mp_.T_pc @ PF_n
    gam = np.zeros(2 * nb)
    gam[nb:nb + n1] = co.eta / co.rho * (mp_.Gc @ pg)        # -(eta/rho) int p_F v.n_c
    gam[:n1] = -co.ctau * (mp_.Gxc @ pg)                     # -c_tau int d_x p_F v_x
    Gblk = sps.block_diag([mp_.Gc, sps.csr_matrix((nb - n1, nb - n1)),
                           sps.csr_matrix((nb, nb))]).tocsr()
    Alin = (co.eta / co.dt) * mp_.Mv + co.nu * co.eta * mp_.S + co.eta * co.beta * Gblk
    g = np.concatenate([interp_mini(mc, mms, "u1", t1), interp_mini(mc, mms, "u2", t1)])
    dmask_u = np.concatenate([mp_.dir_u, mp_.dir_u])
    U = np.where(dmask_u, g, U_n)
    P = P_n.copy()
    dmask = np.concatenate([dmask_u, np.zeros(n1, bool)])
    for it in range(maxit):
        if convection:
            cv, Nm = mini_convection(mc, E, U)
        else:
            cv, Nm = np.zeros(2 * nb), sps.csr_matrix((2 * nb, 2 * nb))
        Fv = Alin @ U - (co.eta / co.dt) * (mp_.Mv @ U_n) + co.eta * cv \
            - co.eta * (mp_.Bq.T @ P) - gam - co.eta * F
        Fq = co.eta * (mp_.Bq @ U)
        J = sps.bmat([[Alin + co.eta * Nm, -co.eta * mp_.Bq.T], [co.eta * mp_.Bq, None]]).tocsr()
        d = _solve_dirichlet(J, -np.concatenate([Fv, Fq]), dmask, np.zeros(len(dmask)))
        U = U + d[:2 * nb]
        P = P + d[2 * nb:]
        if np.linalg.norm(d) <= tol * np.linalg.norm(np.concatenate([U, P])):
            break
    return U, P, it + 1


def algorithm1_mini(N, prm, dt, nsteps, problem="ex1"):
    """Algorithm 1 on one grid of N cells per unit length with MINI + P1;
    returns the problem and the final fields.  problem "ex1": Example 1's
    manufactured solution; "ex3": the Example-3-type variant (Example3)."""
    co = Coefs(prm, dt)
    ex3 = problem == "ex3"
    mms = Example3() if ex3 else MMS(prm)
    mp_ = MiniProblem(N, co, outflow_top=ex3)
    P = [interp_p1(mp_.mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
    U = np.concatenate([interp_mini(mp_.mc, mms, "u1", 0.0), interp_mini(mp_.mc, mms, "u2", 0.0)])
    Pc = interp_p1(mp_.mc, mms, "p", 0.0)
    for n in range(nsteps):
        t1 = (n + 1) * dt
        Pn = mini_porous_step(mp_, mms, P, U, t1)
        U, Pc, _ = mini_ns_step(mp_, mms, U, Pc, P[0], t1, convection=not ex3)
        P = Pn
    return mp_, dict(pF=P[0], pf=P[1], pm=P[2], u=U, p=Pc)


class Example3:
    """Data of the Example-3-type variant (Section 6, Example 3) on the
    two-square geometry: fixed pressures p_F = 1.0e3, p_f = 1.6e3,
    p_m = 4.0e3 on the porous region's outer boundary (Gamma_in, also the
    initial porous state), no sources, a Stokes conduit (no convection)
    whose side walls are cased (no-slip, u = 0) and whose top y = 2 is the
    outflow boundary (T(u, p) n = 0), starting from rest."""
    VALUES = dict(pF=1.0e3, pf=1.6e3, pm=4.0e3)

    def __call__(self, name, xy, tt):
        return np.full(xy.shape[0], self.VALUES.get(name, 0.0))


def example3_params(kF):
    """Section 6, Example 3's parameters (sigma* not given: taken equal to
    sigma) with macro-fracture permeability kF."""
    return dict(phi=[1e-4, 1e-3, 1e-2], C=[1e-4] * 3, k=[kF, 1e-6, 1e-8], mu_tilde=1e-2, sigma=0.5,
                sigma_star=0.5, rho=10.0, alpha=1.0, eta=1.0, nu=1e-2)


def boundary_flux(mesh, U, j):
    """int u_y dx over the conduit lattice row j (a horizontal line; bubbles
    vanish there): the P1 trace integrated exactly (trapezoid)."""
    nb, n1 = n_vel(mesh), mesh.n1
    uy = U[nb + j * n1: nb + (j + 1) * n1]
    return float(mesh.h * (uy[:-1] + uy[1:]).sum() / 2)

def errors(mesh, vec, exact, space):
    """(L2 error, H1-seminorm error) of a P1 ("p1") or MINI ("mini") scalar
    field against exact(X) -> (values (n,), gradients (n, 2))."""
    V, G = (_P1V, np.broadcast_to(_P1G, (len(_WTS), 3, 2))) if space == "p1" else (_MBV, _MBG)
    e2 = g2 = 0.0
    for _, Et, J, det, invJ in _orient(mesh, np.arange(2 * mesh.N ** 2)):
        dofs = mesh.el_p1[Et] if space == "p1" else el_vel(mesh, Et)
        ve = vec[dofs]
        uh = ve @ V.T
        gh = np.einsum("ea,qak->eqk", ve, G @ invJ)
        X = _qp_coords(mesh, Et, J).reshape(-1, 2)
        ux, gx = exact(X)
        w = _WTS * det
        e2 += np.sum(w[None] * (uh - ux.reshape(uh.shape)) ** 2)
        g2 += np.sum(w[None, :, None] * (gh - gx.reshape(gh.shape)) ** 2)
    return np.sqrt(e2), np.sqrt(g2)


# ---------------------------------------------------------------------------
# Algorithm 3 with the paper's elements (Table 1)
# ---------------------------------------------------------------------------
def eval_mini(coarse, vec, X):
    """Values at points X (n, 2) of a MINI (vertices + bubbles) or, with a
    vector of vertex values only, P1 function on the mesh `coarse`."""
    eid, ref = _locate(coarse, X[:, 0], X[:, 1] - coarse.y0)
    val, _ = mini_basis(ref)
    nv = coarse.n1 ** 2
    out = np.einsum("na,na->n", val[:, :3], vec[coarse.el_p1[eid]])
    if len(vec) > nv:
        out += val[:, 3] * vec[nv + eid]
    return out


def prolong_mini(coarse, fine, vec):
    """Reading M5: the fine MINI interpolant of a coarse MINI function."""
    vert = eval_mini(coarse, vec, fine.p1_coords())
    E = np.arange(2 * fine.N ** 2)
    cen = fine.p1_coords()[fine.el_p1[E]].mean(axis=1)
    return np.concatenate([vert, eval_mini(coarse, vec, cen) - vert[fine.el_p1[E]].mean(axis=1)])


def _classify_p1(sd, mesh, outflow_top=False):
    """Per local vertex of Omega_j: 0 free, 1 physical Dirichlet, 2 artificial.
    With outflow_top the conduit's top is natural (Example 3's outflow) and
    only its side walls carry Dirichlet velocity."""
    pn, I, J = sd.p1_nodes(mesh)
    if mesh.region == CONDUIT and outflow_top:
        phys = (I == 0) | (I == mesh.N)
    else:
        phys = (I == 0) | (I == mesh.N) | ((J == 0) if mesh.region == POROUS else (J == mesh.N))
    cls = np.where(sd.artificial_p1(I, J), 2, 0)
    cls[phys] = 1
    return pn, I, J, cls


class MiniOracle2D:
    """Algorithm 3 (Section 5) with MINI + P1: init(), then per step
    coarse_step() and local_step(); merged() reads the corrected fields."""

    def __init__(self, NH, Nh, cuts, overlap, prm, dt, previous="own", problem="ex1"):
        assert Nh % NH == 0 and previous in ("own", "merged")
        self.previous = previous
        self.ex3 = problem == "ex3"
        self.co = Coefs(prm, dt)
        self.mms = Example3() if self.ex3 else MMS(prm)
        self.cg = MiniProblem(NH, self.co, outflow_top=self.ex3)
        self.fg = MiniProblem(Nh, self.co, outflow_top=self.ex3)
        self.subs = make_subdomains(Nh, cuts, overlap)
        self.cuts = cuts
        self.n = 0
        self._cache = {}

    def t(self, n):
        return n * self.co.dt

    def _mesh(self, region):
        return self.fg.mp if region == POROUS else self.fg.mc

    def _pro_u(self, U):
        cm, fm = self.cg.mc, self.fg.mc
        nb = n_vel(cm)
        return np.concatenate([prolong_mini(cm, fm, U[:nb]), prolong_mini(cm, fm, U[nb:])])

    def _pro_p1(self, mesh_c, mesh_f, v):
        return eval_mini(mesh_c, v, mesh_f.p1_coords())

    def init(self):
        cg, fg, mms = self.cg, self.fg, self.mms
        self.P = [interp_p1(cg.mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
        self.U = np.concatenate([interp_mini(cg.mc, mms, "u1", 0.0), interp_mini(cg.mc, mms, "u2", 0.0)])
        self.Pc = interp_p1(cg.mc, mms, "p", 0.0)
        self.P_old, self.U_old = [p.copy() for p in self.P], self.U.copy()
        fineP = [interp_p1(fg.mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
        fineU = np.concatenate([interp_mini(fg.mc, mms, "u1", 0.0), interp_mini(fg.mc, mms, "u2", 0.0)])
        ProlP = [self._pro_p1(cg.mp, fg.mp, p) for p in self.P]
        ProlU = self._pro_u(self.U)
        nb = n_vel(fg.mc)
        self.e = {}
        for sd in self.subs:
            mesh = self._mesh(sd.region)
            pn, _, _, cls = _classify_p1(sd, mesh, self.ex3)
            if sd.region == POROUS:
                self.e[sd.sid] = [np.where(cls == 2, 0.0, fineP[i][pn] - ProlP[i][pn]) for i in range(3)]
            else:
                vi = self._vel_index(sd)
                d = fineU - ProlU
                ev = d[vi]
                ev[self._vel_fixed(sd) == 2] = 0.0
                self.e[sd.sid] = [ev, np.zeros(len(pn))]
        self.n = 0

    def coarse_step(self):
        """Step 1: Algorithm 1's step on T_H."""
        t1 = self.t(self.n + 1)
        self.P_old, self.U_old = [p.copy() for p in self.P], self.U.copy()
        P_new = mini_porous_step(self.cg, self.mms, self.P, self.U, t1)
        U_new, P_c, _ = mini_ns_step(self.cg, self.mms, self.U, self.Pc, self.P[0], t1, convection=not self.ex3)
        self.P, self.U, self.Pc = P_new, U_new, P_c

    # local velocity unknowns of a conduit subdomain: both components of the
    # box's vertices, then of the bubbles of its elements (MINI vector indices)
    def _vel_index(self, sd):
        mesh = self.fg.mc
        nb = n_vel(mesh)
        pn = sd.p1_nodes(mesh)[0]
        E = mesh.elements_in_box(sd.x0, sd.x1, sd.y0, sd.y1)
        one = np.concatenate([pn, mesh.n1 ** 2 + E])
        return np.concatenate([one, nb + one])

    def _vel_fixed(self, sd):
        mesh = self.fg.mc
        _, _, _, cls = _classify_p1(sd, mesh, self.ex3)
        nE = len(mesh.elements_in_box(sd.x0, sd.x1, sd.y0, sd.y1))
        one = np.concatenate([cls, np.zeros(nE, dtype=cls.dtype)])
        return np.concatenate([one, one])

    def local_porous(self, sd, pro):
        """Step 3 (1), Eqs. (5.5)-(5.7) on the P1 space of Omega_j."""
        co, mesh, mms = self.co, self.fg.mp, self.mms
        t1 = self.t(self.n + 1)
        key = ("p", sd.sid)
        if key not in self._cache:
            E = mesh.elements_in_box(sd.x0, sd.x1, sd.y0, sd.y1)
            M, K = p1_mass_stiff(mesh, E)
            G = gamma_p1(mesh, sd.x0, sd.x1)[0] if sd.touches_gamma else None
            self._cache[key] = (E, M, K, G)
        E, M, K, G = self._cache[key]
        pn, _, _, cls = _classify_p1(sd, mesh, self.ex3)
        nn = mesh.n1 ** 2
        PF1, Pf1, Pm1 = pro["P1"]
        PF0, Pf0, Pm0 = pro["P0"]
        Q = [load(mesh, E, lambda X, nm=nm: mms(nm, X, t1), "p1") for nm in ("qF", "qf", "qm")]

        def full(loc):
            v = np.zeros(nn)
            v[pn] = loc
            return v
        eF, ef, em = [full(v) for v in self.e[sd.sid]]
        gam = np.zeros(nn)
        if G is not None:
            nbc, n1c = n_vel(self.fg.mc), self.fg.mc.n1 ** 2
            gam = -G @ (self.fg.T_cp @ pro["U0"][nbc:nbc + n1c])
        rhs = [Q[0] - (co.tau[0] * (M @ (PF1 - PF0)) + co.kap[0] * (K @ PF1) + co.sst * (M @ (PF1 - Pf0)))
               + gam + co.tau[0] * (M @ eF) + co.sst * (M @ ef),
               Q[1] - (co.tau[1] * (M @ (Pf1 - Pf0)) + co.kap[1] * (K @ Pf1) + co.s * (M @ (Pf1 - Pm0))
                       + co.sst * (M @ (Pf1 - PF0)))
               + co.tau[1] * (M @ ef) + co.s * (M @ em) + co.sst * (M @ eF),
               Q[2] - (co.tau[2] * (M @ (Pm1 - Pm0)) + co.kap[2] * (K @ Pm1) + co.s * (M @ (Pm1 - Pf0)))
               + co.tau[2] * (M @ em) + co.s * (M @ ef)]
        A = [(co.tau[0] + co.sst) * M + co.kap[0] * K,
             (co.tau[1] + co.s + co.sst) * M + co.kap[1] * K,
             (co.tau[2] + co.s) * M + co.kap[2] * K]
        xy = mesh.p1_coords()[pn]
        out = []
        for i, nm in enumerate(("pF", "pf", "pm")):
            dvals = np.where(cls == 1, mms(nm, xy, t1) - pro["P1"][i][pn], 0.0)
            out.append(_solve_dirichlet(A[i][pn][:, pn].tocsr(), rhs[i][pn], cls != 0, dvals))
        return out

    def local_conduit(self, sd, pro):
        """Step 3 (2), Eq. (5.8): the Oseen correction on the MINI space of
        Omega_j, linearised about Pi_h u_H^{n+1}."""
        co, mesh, mms = self.co, self.fg.mc, self.mms
        t1 = self.t(self.n + 1)
        E = mesh.elements_in_box(sd.x0, sd.x1, sd.y0, sd.y1)
        key = ("c", sd.sid)
        if key not in self._cache:
            self._cache[key] = mini_stokes(mesh, E)
        Mv, S, Bq = self._cache[key]
        nb, n1 = n_vel(mesh), mesh.n1 ** 2
        W1, W0, Pp = pro["U1"], pro["U0"], pro["Pc1"]
        if self.ex3:
            cv, Nm = np.zeros(2 * nb), sps.csr_matrix((2 * nb, 2 * nb))
        else:
            cv, Nm = mini_convection(mesh, E, W1)
        Gblk = sps.csr_matrix((2 * nb, 2 * nb))
        gam = np.zeros(2 * nb)
        if sd.touches_gamma:
            G, Gx = gamma_p1(mesh, sd.x0, sd.x1)
            Gblk = sps.block_diag([G, sps.csr_matrix((nb - n1, nb - n1)), sps.csr_matrix((nb, nb))]).tocsr()
            pg = self.fg.T_pc @ pro["P0"][0]
            gam[nb:nb + n1] = co.eta / co.rho * (G @ pg)
            gam[:n1] = -co.ctau * (Gx @ pg)
        F = np.concatenate([load(mesh, E, lambda X: mms("f1", X, t1), "mini"),
                            load(mesh, E, lambda X: mms("f2", X, t1), "mini")])
        Avis = co.nu * co.eta * S + co.eta * co.beta * Gblk
        A = (co.eta / co.dt) * Mv + Avis + co.eta * Nm
        vi = self._vel_index(sd)
        fixed = self._vel_fixed(sd)
        pn, I, J, cls = _classify_p1(sd, mesh, self.ex3)
        pfix = sd.artificial_p1(I, J)          # R1p: every artificial vertex, physical ones too
        en = np.zeros(2 * nb)
        en[vi] = self.e[sd.sid][0]
        rv = co.eta * F - ((co.eta / co.dt) * (Mv @ (W1 - W0)) + Avis @ W1
                           - co.eta * (Bq.T @ Pp) + co.eta * cv) + gam + (co.eta / co.dt) * (Mv @ en)
        rq = -co.eta * (Bq @ W1)
        K = sps.bmat([[A[vi][:, vi], -co.eta * Bq.T[vi][:, pn]],
                      [co.eta * Bq[pn][:, vi], None]]).tocsr()
        rhs = np.concatenate([rv[vi], rq[pn]])
        # physical Dirichlet vertices: g(t_{n+1}) - Pi_h u_H^{n+1}
        xyv = mesh.p1_coords()
        nE = len(E)
        g = np.concatenate([mms("u1", xyv[pn], t1), np.zeros(nE), mms("u2", xyv[pn], t1), np.zeros(nE)])
        dv = np.where(fixed == 1, g - W1[vi], 0.0)
        z = _solve_dirichlet(K, rhs, np.concatenate([fixed != 0, pfix]), np.concatenate([dv, np.zeros(len(pn))]))
        return [z[:len(vi)], z[len(vi):]]

    def prolonged(self):
        cg, fg = self.cg, self.fg
        return dict(P1=[self._pro_p1(cg.mp, fg.mp, p) for p in self.P],
                    P0=[self._pro_p1(cg.mp, fg.mp, p) for p in self.P_old],
                    U1=self._pro_u(self.U), U0=self._pro_u(self.U_old),
                    Pc1=self._pro_p1(cg.mc, fg.mc, self.Pc))

    def local_step(self):
        pro = self.prolonged()
        self.e = {sd.sid: (self.local_porous(sd, pro) if sd.region == POROUS else self.local_conduit(sd, pro))
                  for sd in self.subs}
        self.n += 1
        self._pro = pro
        if self.previous == "merged":
            # reading M6: the next step lags the merged correction
            f = self.merged()
            for sd in self.subs:
                mesh = self._mesh(sd.region)
                pn, _, _, cls = _classify_p1(sd, mesh, self.ex3)
                if sd.region == POROUS:
                    self.e[sd.sid] = [np.where(cls == 2, 0.0, (f[k] - pro["P1"][i])[pn])
                                      for i, k in enumerate(("pF", "pf", "pm"))]
                else:
                    vi = self._vel_index(sd)
                    ev = (f["u"] - pro["U1"])[vi]
                    ev[self._vel_fixed(sd) == 2] = 0.0
                    self.e[sd.sid] = [ev, self.e[sd.sid][1]]

    def merged(self):
        """Step 4 (readings R4 and M5): pF, pf, pm (P1), u (MINI), p (P1)."""
        pro = self._pro
        out = {}
        for region in (POROUS, CONDUIT):
            mesh = self._mesh(region)
            i1 = np.arange(mesh.n1)
            vx = 1.0 / owner_counts(self.cuts[(region, 0)], 2 * i1)
            vy = 1.0 / owner_counts(self.cuts[(region, 1)], 2 * i1)
            if region == POROUS:
                acc = [p.copy() for p in pro["P1"]]
            else:
                acc = [pro["U1"].copy(), pro["Pc1"].copy()]
            nb, n1v = n_vel(mesh), mesh.n1 ** 2
            for sd in self.subs:
                if sd.region != region:
                    continue
                dx0, dx1, dy0, dy1 = sd.d
                pn, I, J, _ = _classify_p1(sd, mesh, self.ex3)
                inD = (I >= dx0) & (I <= dx1) & (J >= dy0) & (J <= dy1)
                w = vx[I] * vy[J]
                if region == POROUS:
                    for k in range(3):
                        acc[k][pn[inD]] += w[inD] * self.e[sd.sid][k][inD]
                    continue
                E = mesh.elements_in_box(sd.x0, sd.x1, sd.y0, sd.y1)
                cell = mesh.el_cell[E]
                inDe = (cell[:, 0] >= dx0) & (cell[:, 0] < dx1) & (cell[:, 1] >= dy0) & (cell[:, 1] < dy1)
                ev = self.e[sd.sid][0]
                nloc = len(pn) + len(E)
                for c in range(2):
                    part = ev[c * nloc:(c + 1) * nloc]
                    acc[0][c * nb + pn[inD]] += w[inD] * part[:len(pn)][inD]
                    acc[0][c * nb + n1v + E[inDe]] += part[len(pn):][inDe]
                acc[1][pn[inD]] += w[inD] * self.e[sd.sid][1][inD]
            if region == POROUS:
                out["pF"], out["pf"], out["pm"] = acc
            else:
                out["u"], out["p"] = acc
        return out
