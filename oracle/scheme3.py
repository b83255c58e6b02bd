"""Algorithm 1 (Section 3.3, partitioned time stepping) and Algorithm 3 (the
two-grid local parallel method, Section 5) in 3D, plain FP64 with
scipy.sparse direct solves, on the unit-cube regions of mesh3 (porous
(0,1)^3 below the conduit (0,1)^2 x (1,2), Gamma at z = 1, n_c = (0,0,-1)).

Notation and readings as in scheme.py (the 2D oracle): tau_i = phi_i C_i / dt,
kappa_i = k_i / mu_tilde, s* = sigma* k_f / mu_tilde, s = sigma k_m / mu_tilde,
the Beavers-Joseph coefficient beta = alpha nu / sqrt(k_F) (with Pi = k_F I and
d = 3 the paper's alpha nu sqrt(d) / sqrt(trace Pi) is the same number),
c_tau = eta nu alpha sqrt(k_F) / mu_tilde; the Navier-Stokes step is fully
implicit, solved by Newton's method to a relative update <= 1e-13; initial
data are nodal interpolants.  In 3D v . n_c = -v_z and P_tau v = (v_x, v_y).
"""
import numpy as np
import scipy.sparse as sps

from . import forms3
from .fe3 import p1_basis3, p2_basis3
from .mesh import owner_counts
from .mesh3 import RegionMesh3, POROUS, CONDUIT, PERMS, make_subdomains3
from .mms3 import MMS3
from .scheme import Coefs, _solve_dirichlet


def region_dirichlet_p2_3d(mesh):
    """Physical boundary of a whole region (its boundary minus Gamma)."""
    L = mesh.n2
    q = np.arange(L ** 3)
    a, b, c = q % L, (q // L) % L, q // (L * L)
    N2 = 2 * mesh.N
    d = (a == 0) | (a == N2) | (b == 0) | (b == N2)
    d |= (c == 0) if mesh.region == POROUS else (c == N2)
    return d


def interp(mesh, mms, name, tt, p1=False):
    return mms(name, mesh.p1_coords() if p1 else mesh.p2_coords(), tt)


class GridProblem3:
    """Constant operators of one grid (porous + conduit regions of N^3 cells)."""

    def __init__(self, N, co):
        self.mp = RegionMesh3(N, POROUS)
        self.mc = RegionMesh3(N, CONDUIT)
        self.co = co
        allel = np.arange(6 * N ** 3)
        self.M, self.K = forms3.p2_mass_stiff(self.mp, allel)
        self.Mv, self.S, self.Bq = forms3.stokes_blocks(self.mc, allel)
        self.Gp, _, _ = forms3.gamma_forms(self.mp)
        self.Gc, self.Gxc, self.Gyc = forms3.gamma_forms(self.mc)
        self.T_cp = forms3.gamma_transfer(self.mc, self.mp)
        self.T_pc = forms3.gamma_transfer(self.mp, self.mc)
        self.dir_p = region_dirichlet_p2_3d(self.mp)
        self.dir_c = region_dirichlet_p2_3d(self.mc)


def porous_step3(gp, mms, P_n, U_n, t1):
    """The three decoupled SPD solves of Algorithm 1's porous step with lagged
    exchange and the lagged Gamma flux u^n . n_c = -u_z^n."""
    co, M, K = gp.co, gp.M, gp.K
    n2 = gp.mc.n2 ** 3
    PF, Pf, Pm = P_n
    xyz = gp.mp.p2_coords()
    E = np.arange(6 * gp.mp.N ** 3)
    Q = [forms3.load_p2(gp.mp, E, lambda X, nm=nm: mms(nm, X, t1)) for nm in ("qF", "qf", "qm")]
    gam = -gp.Gp @ (gp.T_cp @ U_n[2 * n2:])
    A = [(co.tau[0] + co.sst) * M + co.kap[0] * K,
         (co.tau[1] + co.s + co.sst) * M + co.kap[1] * K,
         (co.tau[2] + co.s) * M + co.kap[2] * K]
    rhs = [Q[0] + co.tau[0] * (M @ PF) + co.sst * (M @ Pf) + gam,
           Q[1] + co.tau[1] * (M @ Pf) + co.s * (M @ Pm) + co.sst * (M @ PF),
           Q[2] + co.tau[2] * (M @ Pm) + co.s * (M @ Pf)]
    out = []
    for i, nm in enumerate(("pF", "pf", "pm")):
        out.append(_solve_dirichlet(A[i], rhs[i], gp.dir_p, mms(nm, xyz, t1)))
    return out


def conduit_gamma_rhs3(gp, PF_n, co):
    """Right-hand-side Gamma terms of the conduit equation:
    -(eta/rho) int p_F v . n_c - c_tau int grad_tau p_F . P_tau v, with
    v . n_c = -v_z."""
    n2 = gp.mc.n2 ** 3
    pg = gp.T_pc @ PF_n
    r = np.zeros(3 * n2)
    r[2 * n2:] = co.eta / co.rho * (gp.Gc @ pg)
    r[:n2] = -co.ctau * (gp.Gxc @ pg)
    r[n2:2 * n2] = -co.ctau * (gp.Gyc @ pg)
    return r


def ns_step3(gp, mms, U_n, P_n, PF_n, t1, tol=1e-13, maxit=30, convection=True):
    """Algorithm 1's fully implicit backward-Euler Navier-Stokes step with
    lagged p_F on Gamma, solved by Newton's method."""
    co, mc = gp.co, gp.mc
    n2, n1 = mc.n2 ** 3, mc.n1 ** 3
    E = np.arange(6 * mc.N ** 3)
    F = np.concatenate([forms3.load_p2(mc, E, lambda X, c=c: mms("f%d" % (c + 1), X, t1)) for c in range(3)])
    gam = conduit_gamma_rhs3(gp, PF_n, co)
    Gblk = sps.block_diag([gp.Gc, gp.Gc, sps.csr_matrix((n2, n2))]).tocsr()
    Alin = (co.eta / co.dt) * gp.Mv + co.nu * co.eta * gp.S + co.eta * co.beta * Gblk
    xyz = mc.p2_coords()
    g = np.concatenate([mms("u%d" % (c + 1), xyz, t1) for c in range(3)])
    dmask_u = np.concatenate([gp.dir_c] * 3)
    U = np.where(dmask_u, g, U_n).astype(np.float64)
    P = P_n.copy()
    dmask = np.concatenate([dmask_u, np.zeros(n1, bool)])
    for it in range(maxit):
        if convection:
            cv, Nm = forms3.convection(mc, E, U)
        else:
            cv, Nm = np.zeros(3 * n2), sps.csr_matrix((3 * n2, 3 * n2))
        Fv = Alin @ U - (co.eta / co.dt) * (gp.Mv @ U_n) + co.eta * cv \
            - co.eta * (gp.Bq.T @ P) - gam - co.eta * F
        Fq = co.eta * (gp.Bq @ U)
        J = sps.bmat([[Alin + co.eta * Nm, -co.eta * gp.Bq.T], [co.eta * gp.Bq, None]]).tocsr()
        d = _solve_dirichlet(J, -np.concatenate([Fv, Fq]), dmask, np.zeros(len(dmask)))
        U = U + d[:3 * n2]
        P = P + d[3 * n2:]
        if np.linalg.norm(d) <= tol * np.linalg.norm(np.concatenate([U, P])):
            break
    return U, P, it + 1


def algorithm1_3d(N, prm, dt, nsteps, convection=True):
    """Algorithm 1 on one grid of N^3 cells per region; returns the grid and
    the final fields."""
    co = Coefs(prm, dt)
    mms = MMS3(prm)
    gp = GridProblem3(N, co)
    P = [interp(gp.mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
    U = np.concatenate([interp(gp.mc, mms, "u%d" % (c + 1), 0.0) for c in range(3)])
    Pc = interp(gp.mc, mms, "p", 0.0, p1=True)
    for n in range(nsteps):
        t1 = (n + 1) * dt
        Pn = porous_step3(gp, mms, P, U, t1)
        U, Pc, _ = ns_step3(gp, mms, U, Pc, P[0], t1, convection=convection)
        P = Pn
    return gp, dict(pF=P[0], pf=P[1], pm=P[2], u=U, p=Pc)


# ---------------------------------------------------------------------------
# exact prolongation between nested Kuhn meshes (coarse element polynomial
# evaluated at fine nodes)
# ---------------------------------------------------------------------------
def _locate3(coarse, X):
    """Coarse element containing region-relative points X (n, 3) and their
    reference coordinates.  A point lies in the Kuhn tetrahedron of the
    permutation that sorts its in-cell coordinates in decreasing order."""
    H, NH = coarse.h, coarse.N
    idx = np.minimum((X / H).astype(np.int64), NH - 1)
    loc = X - idx * H
    order = np.argsort(-loc, axis=1, kind="stable")
    rank = np.array([PERMS.index(tuple(o)) for o in order])
    cell = idx[:, 0] + NH * (idx[:, 1] + NH * idx[:, 2])
    eid = 6 * cell + rank
    ref = np.zeros_like(X)
    for r in range(6):
        sel = rank == r
        if sel.any():
            ref[sel] = loc[sel] @ np.linalg.inv(coarse.jacobian(r)).T
    return eid, ref


def prolong_p2_3d(coarse, fine, vec):
    c = fine.p2_coords()
    X = c - np.array([0.0, 0.0, fine.z0])
    eid, ref = _locate3(coarse, X)
    val, _ = p2_basis3(ref)
    return np.einsum("na,na->n", val, vec[coarse.el_p2[eid]])


def prolong_p1_3d(coarse, fine, vec):
    c = fine.p1_coords()
    X = c - np.array([0.0, 0.0, fine.z0])
    eid, ref = _locate3(coarse, X)
    val, _ = p1_basis3(ref)
    return np.einsum("na,na->n", val, vec[coarse.el_p1[eid]])


# ---------------------------------------------------------------------------
# Algorithm 3, Steps 2-4, in 3D
# ---------------------------------------------------------------------------
def prolong_u_3d(coarse, fine, vec):
    """Component-blocked P2 velocity from the coarse to the fine lattice."""
    n2c = coarse.n2 ** 3
    return np.concatenate([prolong_p2_3d(coarse, fine, vec[c * n2c:(c + 1) * n2c]) for c in range(3)])


def conduit_gamma_rhs3_box(gp, PF_n, co, G, Gx, Gy):
    """conduit_gamma_rhs3 with the Gamma forms of one box's interface triangles."""
    n2 = gp.mc.n2 ** 3
    pg = gp.T_pc @ PF_n
    r = np.zeros(3 * n2)
    r[2 * n2:] = co.eta / co.rho * (G @ pg)
    r[:n2] = -co.ctau * (Gx @ pg)
    r[n2:2 * n2] = -co.ctau * (Gy @ pg)
    return r


class Oracle3D:
    """Algorithm 3 in 3D, the same steps and readings as the 2D oracle
    (Oracle2D) on the Kuhn meshes: init() once, then per time step
    coarse_step() and local_step(); merged() and coarse() read results.
    cuts: {(region, axis): [0, ..., Nh]} for axes 0, 1, 2 (x, y, vertical),
    overlap in fine cells (an int or a per-axis triple)."""

    def __init__(self, NH, Nh, cuts, overlap, prm, dt, convection=True):
        assert Nh % NH == 0
        self.co = Coefs(prm, dt)
        self.mms = MMS3(prm)
        self.cg = GridProblem3(NH, self.co)
        self.fg = GridProblem3(Nh, self.co)
        self.subs = make_subdomains3(Nh, cuts, overlap)
        self.cuts = cuts
        self.convection = convection
        self.n = 0
        self._cache = {}

    def t(self, n):
        return n * self.co.dt

    def _fine_mesh(self, region):
        return self.fg.mp if region == POROUS else self.fg.mc

    def init(self):
        """Nodal interpolants at t = 0 on both grids; e_j^0 = I_h x_0 - Pi_h x_H^0
        on each Omega_j, zero on artificial faces (pressure corrections zero)."""
        cg, fg, mms = self.cg, self.fg, self.mms
        self.P = [interp(cg.mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
        self.U = np.concatenate([interp(cg.mc, mms, "u%d" % (c + 1), 0.0) for c in range(3)])
        self.Pc = interp(cg.mc, mms, "p", 0.0, p1=True)
        self.P_old, self.U_old = [p.copy() for p in self.P], self.U.copy()
        fineP = [interp(fg.mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
        fineU = np.concatenate([interp(fg.mc, mms, "u%d" % (c + 1), 0.0) for c in range(3)])
        ProlP = [prolong_p2_3d(cg.mp, fg.mp, p) for p in self.P]
        ProlU = prolong_u_3d(cg.mc, fg.mc, self.U)
        n2f = fg.mc.n2 ** 3
        self.e = {}
        for sd in self.subs:
            mesh = self._fine_mesh(sd.region)
            nodes = sd.p2_nodes(mesh)[0]
            cls = sd.classify_p2(mesh)
            if sd.region == POROUS:
                vals = [np.where(cls == 2, 0.0, fineP[i][nodes] - ProlP[i][nodes]) for i in range(3)]
            else:
                vals = [np.where(cls == 2, 0.0, fineU[c * n2f + nodes] - ProlU[c * n2f + nodes]) for c in range(3)]
                vals.append(np.zeros(len(sd.p1_nodes(mesh)[0])))
            self.e[sd.sid] = vals
        self.n = 0

    # -- Step 1
    def coarse_step(self):
        t1 = self.t(self.n + 1)
        self.P_old, self.U_old = [p.copy() for p in self.P], self.U.copy()
        P_new = porous_step3(self.cg, self.mms, self.P, self.U, t1)
        U_new, P_c, self.newton_its = ns_step3(self.cg, self.mms, self.U, self.Pc, self.P[0], t1,
                                               convection=self.convection)
        self.P, self.U, self.Pc = P_new, U_new, P_c

    def _box_elements(self, mesh, sd):
        return mesh.elements_in_box(sd.x0, sd.x1, sd.y0, sd.y1, sd.z0, sd.z1)

    # -- Step 3 (1): Eqs. (5.5)-(5.7)
    def local_porous(self, sd, pro):
        co, mesh, mms = self.co, self.fg.mp, self.mms
        t1 = self.t(self.n + 1)
        key = ("p", sd.sid)
        if key not in self._cache:
            E = self._box_elements(mesh, sd)
            M, K = forms3.p2_mass_stiff(mesh, E)
            G = forms3.gamma_forms(mesh, sd.x0, sd.x1, sd.y0, sd.y1)[0] if sd.touches_gamma else None
            self._cache[key] = (E, M, K, G)
        E, M, K, G = self._cache[key]
        nodes = sd.p2_nodes(mesh)[0]
        cls = sd.classify_p2(mesh)
        nn = mesh.n2 ** 3
        PF1, Pf1, Pm1 = pro["P1"]
        PF0, Pf0, Pm0 = pro["P0"]
        Q = [forms3.load_p2(mesh, E, lambda X, nm=nm: mms(nm, X, t1)) for nm in ("qF", "qf", "qm")]

        def full(loc):
            v = np.zeros(nn)
            v[nodes] = loc
            return v
        eF, ef, em = [full(v) for v in self.e[sd.sid]]
        gam = np.zeros(nn)
        if G is not None:
            n2c = self.fg.mc.n2 ** 3
            gam = -G @ (self.fg.T_cp @ pro["U0"][2 * n2c:])     # + <u_cH^n . n_c, v_F>, v . n_c = -v_z
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
        xyz = mesh.p2_coords()[nodes]
        out = []
        for i, nm in enumerate(("pF", "pf", "pm")):
            dvals = np.where(cls == 1, mms(nm, xyz, t1) - pro["P1"][i][nodes], 0.0)
            out.append(_solve_dirichlet(A[i][nodes][:, nodes].tocsr(), rhs[i][nodes], cls != 0, dvals))
        return out

    # -- Step 3 (2): Eq. (5.8)
    def local_conduit(self, sd, pro):
        co, mesh, mms = self.co, self.fg.mc, self.mms
        t1 = self.t(self.n + 1)
        E = self._box_elements(mesh, sd)
        Mv, S, Bq = forms3.stokes_blocks(mesh, E)
        n2 = mesh.n2 ** 3
        W1, W0, Pp = pro["U1"], pro["U0"], pro["Pc1"]
        if self.convection:
            cv, Nm = forms3.convection(mesh, E, W1)
        else:
            cv, Nm = np.zeros(3 * n2), sps.csr_matrix((3 * n2, 3 * n2))
        if sd.touches_gamma:
            G, Gx, Gy = forms3.gamma_forms(mesh, sd.x0, sd.x1, sd.y0, sd.y1)
            Gblk = sps.block_diag([G, G, sps.csr_matrix((n2, n2))]).tocsr()
            gam = conduit_gamma_rhs3_box(self.fg, pro["P0"][0], co, G, Gx, Gy)
        else:
            Gblk = sps.csr_matrix((3 * n2, 3 * n2))
            gam = np.zeros(3 * n2)
        F = np.concatenate([forms3.load_p2(mesh, E, lambda X, c=c: mms("f%d" % (c + 1), X, t1)) for c in range(3)])
        Avis = co.nu * co.eta * S + co.eta * co.beta * Gblk
        A = (co.eta / co.dt) * Mv + Avis + co.eta * Nm
        nodes = sd.p2_nodes(mesh)[0]
        pn, I, J, K = sd.p1_nodes(mesh)
        cls = sd.classify_p2(mesh)
        pfix = sd.artificial_p1(I, J, K)
        en = np.zeros(3 * n2)
        for c in range(3):
            en[c * n2 + nodes] = self.e[sd.sid][c]
        rv = co.eta * F - ((co.eta / co.dt) * (Mv @ (W1 - W0)) + Avis @ W1
                           - co.eta * (Bq.T @ Pp) + co.eta * cv) + gam + (co.eta / co.dt) * (Mv @ en)
        rq = -co.eta * (Bq @ W1)
        vi = np.concatenate([c * n2 + nodes for c in range(3)])
        Kmat = sps.bmat([[A[vi][:, vi], -co.eta * Bq.T[vi][:, pn]],
                         [co.eta * Bq[pn][:, vi], None]]).tocsr()
        rhs = np.concatenate([rv[vi], rq[pn]])
        xyz = mesh.p2_coords()[nodes]
        dv = [np.where(cls == 1, mms("u%d" % (c + 1), xyz, t1) - W1[c * n2 + nodes], 0.0) for c in range(3)]
        dmask = np.concatenate([cls != 0, cls != 0, cls != 0, pfix])
        dvals = np.concatenate(dv + [np.zeros(len(pn))])
        z = _solve_dirichlet(Kmat, rhs, dmask, dvals)
        nv = len(nodes)
        return [z[:nv], z[nv:2 * nv], z[2 * nv:3 * nv], z[3 * nv:]]

    # -- Steps 3 and 4
    def prolonged(self):
        cg, fg = self.cg, self.fg
        return dict(P1=[prolong_p2_3d(cg.mp, fg.mp, p) for p in self.P],
                    P0=[prolong_p2_3d(cg.mp, fg.mp, p) for p in self.P_old],
                    U1=prolong_u_3d(cg.mc, fg.mc, self.U),
                    U0=prolong_u_3d(cg.mc, fg.mc, self.U_old),
                    Pc1=prolong_p1_3d(cg.mc, fg.mc, self.Pc))

    def local_step(self):
        pro = self.prolonged()
        self.e = {sd.sid: (self.local_porous(sd, pro) if sd.region == POROUS else self.local_conduit(sd, pro))
                  for sd in self.subs}
        self.n += 1
        self._pro = pro
        return pro

    def merged(self):
        """Step 4 with the partition-of-unity weights of the 2D oracle, one
        factor per axis: w = 1 / (owners along x) (owners along y) (owners
        along the vertical) of the closed cores."""
        pro = self._pro
        out = {}
        for region in (POROUS, CONDUIT):
            mesh = self._fine_mesh(region)
            a = np.arange(mesh.n2)
            i1 = np.arange(mesh.n1)
            w2 = [1.0 / owner_counts(self.cuts[(region, ax)], a) for ax in range(3)]
            w1 = [1.0 / owner_counts(self.cuts[(region, ax)], 2 * i1) for ax in range(3)]
            n2 = mesh.n2 ** 3
            if region == POROUS:
                acc = [p.copy() for p in pro["P1"]]
            else:
                acc = [pro["U1"][c * n2:(c + 1) * n2].copy() for c in range(3)] + [pro["Pc1"].copy()]
            for sd in self.subs:
                if sd.region != region:
                    continue
                d = sd.d
                nodes, A, B, C = sd.p2_nodes(mesh)
                inD = ((A >= 2 * d[0]) & (A <= 2 * d[1]) & (B >= 2 * d[2]) & (B <= 2 * d[3])
                       & (C >= 2 * d[4]) & (C <= 2 * d[5]))
                w = w2[0][A] * w2[1][B] * w2[2][C]
                nv = 3
                for k in range(nv):
                    acc[k][nodes[inD]] += w[inD] * self.e[sd.sid][k][inD]
                if region == CONDUIT:
                    pn, I, J, K = sd.p1_nodes(mesh)
                    inDp = ((I >= d[0]) & (I <= d[1]) & (J >= d[2]) & (J <= d[3]) & (K >= d[4]) & (K <= d[5]))
                    wp = w1[0][I] * w1[1][J] * w1[2][K]
                    acc[3][pn[inDp]] += wp[inDp] * self.e[sd.sid][3][inDp]
            if region == POROUS:
                out["pF"], out["pf"], out["pm"] = acc
            else:
                out["u"] = np.concatenate(acc[:3])
                out["p"] = acc[3]
        return out

    def coarse(self):
        return dict(pF=self.P[0], pf=self.P[1], pm=self.P[2], u=self.U, p=self.Pc)
