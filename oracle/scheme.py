"""Algorithm 3 (Section 5, "Local Parallel Finite Element Algorithm") in plain
FP64 with scipy.sparse direct solves, plus Algorithm 1 (Section 3.3) on any
single grid.

Notation follows the paper: tau_i = phi_i C_i / dt, kappa_i = k_i / mu_tilde,
s* = sigma* k_f / mu_tilde (F-f exchange), s = sigma k_m / mu_tilde (f-m
exchange), beta = alpha nu / sqrt(k_F) (Beavers-Joseph; sqrt(d)/sqrt(tr Pi)
with Pi = k_F I), c_tau = eta nu alpha sqrt(k_F) / mu_tilde.  Gamma is y = 1 with
n_c = (0, -1), so v . n_c = -v_y and P_tau v = v_x.

Readings of points the paper leaves open (kept identical in the HIP library):
  R1  local correction spaces vanish on the artificial boundary of Omega_j;
      Gamma stays natural; a node on both an artificial face and the physical
      boundary takes the physical value.
  R2  on the physical boundary the correction equals g(t_{n+1}) - Pi_h x_H^{n+1}.
  R1p the pressure correction and its test functions vanish on the artificial
      boundary too (the pressure analogue of R1, the compact-support space
      Q_0^h used in the local a priori estimate of Section 5.1).  Every test
      function of a local problem is then supported inside Omega_j, so the
      coarse-residual terms equal the global fine residual there, H = h gives
      zero corrections, and no pressure gauge is needed (the constant mode is
      excluded by the zero artificial-face values).
  R4  merge: x_h = Pi_h x_H + sum_j w_j e_j, w_j = 1 / #{closed D_k containing
      the node}, summed in ascending j.
  R5  the coarse Navier-Stokes step is solved by Newton's method to a relative
      update <= 1e-13 (the fully implicit scheme of Step 1 (2)).
  R6  convective trilinear form ((u.grad)u, v), as written in Section 3.1.
  R7  initial data by nodal interpolation on both grids.
  R8  typos: p_Fh^{n+1} -> p_FH^{n+1} in the bracket of (5.5); xi_{fh,j}^n ->
      e_{fh,j}^n in (5.7); p_cH -> p_H in (5.8).
  R17 time levels as written: porous Gamma flux uses u_cH^n, conduit uses p_FH^n;
      sources and Dirichlet data at t_{n+1} = (n+1) dt.
  R18 the lagged e^n of Eqs. (5.5)-(5.8) is the subdomain's own e_j^n, as the
      equations write it (previous="own"); previous="merged" lags instead the
      merged correction of Step 4 restricted to Omega_j (zero on its
      artificial faces; the pressure correction is not lagged), the reading
      under which the paper's Table 1 porous errors are reproduced with its
      own elements.
"""
import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from . import forms
from .fe import p2_basis, p1_basis
from .mesh import RegionMesh, POROUS, CONDUIT, make_subdomains, owner_counts
from .mms import MMS

FIELDS = ("u", "p", "pF", "pf", "pm")


class Coefs:
    def __init__(self, prm, dt):
        mu = prm["mu_tilde"]
        kF, kf, km = prm["k"]
        self.tau = [prm["phi"][i] * prm["C"][i] / dt for i in range(3)]
        self.kap = [kF / mu, kf / mu, km / mu]
        self.sst = prm["sigma_star"] * kf / mu
        self.s = prm["sigma"] * km / mu
        self.eta, self.nu, self.rho = prm["eta"], prm["nu"], prm["rho"]
        self.dt = dt
        self.beta = prm["alpha"] * prm["nu"] / np.sqrt(kF)
        self.ctau = prm["eta"] * prm["nu"] * prm["alpha"] * np.sqrt(kF) / mu


# ---------------------------------------------------------------------------
# interpolation and exact prolongation between nested grids
# ---------------------------------------------------------------------------
def interp_p2(mesh, mms, name, tt):
    return mms(name, mesh.p2_coords(), tt)


def interp_p1(mesh, mms, name, tt):
    return mms(name, mesh.p1_coords(), tt)


def _locate(coarse, X, Y):
    """Coarse element containing region-relative points (X, Y) and its
    reference coordinates."""
    H, NH = coarse.h, coarse.N
    i = np.minimum((X / H).astype(np.int64), NH - 1)
    j = np.minimum((Y / H).astype(np.int64), NH - 1)
    lx, ly = X - i * H, Y - j * H
    t = (ly > lx + 1e-12 * H).astype(np.int64)            # T1 above the diagonal
    eid = 2 * (i + NH * j) + t
    ref = np.zeros((len(X), 2))
    for o in (0, 1):
        sel = t == o
        Jinv = np.linalg.inv(coarse.jacobian(o))
        ref[sel] = (np.stack([lx[sel], ly[sel]], 1)) @ Jinv.T
    return eid, ref


def prolong_p2(coarse, fine, vec):
    """Pi_h: evaluate a coarse P2 function at fine P2 nodes (exact for nested grids)."""
    c = fine.p2_coords()
    eid, ref = _locate(coarse, c[:, 0], c[:, 1] - fine.y0)
    val, _ = p2_basis(ref)
    return np.einsum("na,na->n", val, vec[coarse.el_p2[eid]])


def prolong_p1(coarse, fine, vec):
    c = fine.p1_coords()
    eid, ref = _locate(coarse, c[:, 0], c[:, 1] - fine.y0)
    val, _ = p1_basis(ref)
    return np.einsum("na,na->n", val, vec[coarse.el_p1[eid]])


def prolong_u(coarse, fine, U):
    n = coarse.n2 ** 2
    return np.concatenate([prolong_p2(coarse, fine, U[:n]), prolong_p2(coarse, fine, U[n:])])


# ---------------------------------------------------------------------------
# Dirichlet sets of a whole region (physical boundary minus Gamma)
# ---------------------------------------------------------------------------
def region_dirichlet_p2(mesh):
    c = np.arange(mesh.n2 ** 2)
    a, b = c % mesh.n2, c // mesh.n2
    N2 = 2 * mesh.N
    d = (a == 0) | (a == N2)
    d |= (b == 0) if mesh.region == POROUS else (b == N2)
    return d


def _solve_dirichlet(A, rhs, dmask, dvals):
    """Solve rows/cols of free dofs of A z = rhs with z = dvals on dmask."""
    free = ~dmask
    z = np.where(dmask, dvals, 0.0)
    r = rhs[free] - A[free][:, dmask] @ z[dmask]
    Aff = A[free][:, free].tocsc()
    z[free] = spla.spsolve(Aff, r)
    return z


# ---------------------------------------------------------------------------
# Algorithm 1 / Algorithm 3 Step 1 on one grid (porous part: Eqs. (5.1)-(5.3))
# ---------------------------------------------------------------------------
class GridProblem:
    """Constant operators of one grid (porous + conduit regions of size N)."""

    def __init__(self, N, co):
        self.mp = RegionMesh(N, POROUS)
        self.mc = RegionMesh(N, CONDUIT)
        self.co = co
        allp = np.arange(2 * N * N)
        self.M, self.K = forms.p2_mass_stiff(self.mp, allp)
        self.Mv, self.S, self.Bq = forms.stokes_blocks(self.mc, allp)
        self.Gp, _ = forms.gamma_forms(self.mp)
        self.Gc, self.Gxc = forms.gamma_forms(self.mc)
        self.T_cp = forms.gamma_transfer(self.mc, self.mp)
        self.T_pc = forms.gamma_transfer(self.mp, self.mc)
        self.dir_p = region_dirichlet_p2(self.mp)
        self.dir_c = region_dirichlet_p2(self.mc)


def porous_step(gp, mms, P_n, U_n, t1):
    """Eqs. (5.1)-(5.3) (= Algorithm 1 Step 1 on the same grid): three decoupled
    SPD solves with lagged exchange and lagged Gamma flux u^n . n_c."""
    co, M, K = gp.co, gp.M, gp.K
    n2 = gp.mc.n2 ** 2
    PF, Pf, Pm = P_n
    xy = gp.mp.p2_coords()
    E = np.arange(2 * gp.mp.N ** 2)
    Q = [forms.load_p2(gp.mp, E, lambda X, nm=nm: mms(nm, X, t1)) for nm in ("qF", "qf", "qm")]
    # -int_Gamma v_F u^n.n_c moved to the right: + int v_F (u.n_c) = - int v_F u_y
    gam = -gp.Gp @ (gp.T_cp @ U_n[n2:])
    A = [(co.tau[0] + co.sst) * M + co.kap[0] * K,
         (co.tau[1] + co.s + co.sst) * M + co.kap[1] * K,
         (co.tau[2] + co.s) * M + co.kap[2] * K]
    rhs = [Q[0] + co.tau[0] * (M @ PF) + co.sst * (M @ Pf) + gam,
           Q[1] + co.tau[1] * (M @ Pf) + co.s * (M @ Pm) + co.sst * (M @ PF),
           Q[2] + co.tau[2] * (M @ Pm) + co.s * (M @ Pf)]
    out = []
    for i, nm in enumerate(("pF", "pf", "pm")):
        g = mms(nm, xy, t1)
        out.append(_solve_dirichlet(A[i], rhs[i], gp.dir_p, g))
    return out


def conduit_gamma_rhs(gp, PF_n, co, mesh=None, G=None, Gx=None):
    """Right-hand-side Gamma terms of the conduit equation moved to the right:
    -(eta/rho) int p_F v.n_c - c_tau int d_x p_F v_x  (v.n_c = -v_y)."""
    mc = gp.mc if mesh is None else mesh
    G = gp.Gc if G is None else G
    Gx = gp.Gxc if Gx is None else Gx
    n2 = mc.n2 ** 2
    pg = gp.T_pc @ PF_n
    r = np.zeros(2 * n2)
    r[n2:] = co.eta / co.rho * (G @ pg)
    r[:n2] = -co.ctau * (Gx @ pg)
    return r


def ns_step(gp, mms, U_n, P_n, PF_n, t1, tol=1e-13, maxit=30, convection=True):
    """Eq. (5.4) (= Algorithm 1 Step 2): fully implicit backward Euler
    Navier-Stokes with lagged p_F on Gamma, solved by Newton's method."""
    co, mc = gp.co, gp.mc
    n2, n1 = mc.n2 ** 2, mc.n1 ** 2
    E = np.arange(2 * mc.N ** 2)
    F = np.concatenate([forms.load_p2(mc, E, lambda X: mms("f1", X, t1)),
                        forms.load_p2(mc, E, lambda X: mms("f2", X, t1))])
    gam = conduit_gamma_rhs(gp, PF_n, co)
    Gblk = sps.block_diag([gp.Gc, sps.csr_matrix((n2, n2))]).tocsr()
    Alin = (co.eta / co.dt) * gp.Mv + co.nu * co.eta * gp.S + co.eta * co.beta * Gblk
    xy = mc.p2_coords()
    g = np.concatenate([mms("u1", xy, t1), mms("u2", xy, t1)])
    dmask_u = np.concatenate([gp.dir_c, gp.dir_c])
    U = np.where(dmask_u, g, U_n).astype(np.float64)
    P = P_n.copy()
    dmask = np.concatenate([dmask_u, np.zeros(n1, bool)])
    for it in range(maxit):
        if convection:
            cv, Nm = forms.convection(mc, E, U)
        else:
            cv, Nm = np.zeros(2 * n2), sps.csr_matrix((2 * n2, 2 * n2))
        Fv = Alin @ U - (co.eta / co.dt) * (gp.Mv @ U_n) + co.eta * cv \
            - co.eta * (gp.Bq.T @ P) - gam - co.eta * F
        Fq = co.eta * (gp.Bq @ U)
        J = sps.bmat([[Alin + co.eta * Nm, -co.eta * gp.Bq.T], [co.eta * gp.Bq, None]]).tocsr()
        rhs = -np.concatenate([Fv, Fq])
        d = _solve_dirichlet(J, rhs, dmask, np.zeros(len(dmask)))
        U = U + d[:2 * n2]
        P = P + d[2 * n2:]
        x = np.concatenate([U, P])
        if np.linalg.norm(d) <= tol * np.linalg.norm(x):
            break
    return U, P, it + 1


# ---------------------------------------------------------------------------
# Algorithm 3, Steps 2-4
# ---------------------------------------------------------------------------
class Oracle2D:
    """Algorithm 3 in 2D.  Call sequence: init() once, then per time step
    coarse_step() followed by local_step(); merged(), coarse(), local() read
    results.

    NH, Nh: coarse and fine cells per unit length (Nh a multiple of NH).
    cuts: {(region, axis): [0, ..., Nh]} core cut lattices in fine cells.
    overlap: enlargement of D_j in fine cells.  prm: model parameters.
    """

    def __init__(self, NH, Nh, cuts, overlap, prm, dt, convection=True, previous="own"):
        assert Nh % NH == 0 and previous in ("own", "merged")
        self.previous = previous
        self.co = Coefs(prm, dt)
        self.mms = MMS(prm)
        self.cg = GridProblem(NH, self.co)
        self.fg = GridProblem(Nh, self.co)
        self.subs = make_subdomains(Nh, cuts, overlap)
        self.cuts = cuts
        self.convection = convection
        self.n = 0
        self._cache = {}

    # -- helpers ------------------------------------------------------------
    def t(self, n):
        return n * self.co.dt

    def _fine_mesh(self, region):
        return self.fg.mp if region == POROUS else self.fg.mc

    def init(self):
        """Coarse nodal interpolants of the exact data at t = 0 and the initial
        corrections e_j^0 = I_h x_0 - Pi_h x_H^0 (0 on artificial faces)."""
        cg, fg, mms = self.cg, self.fg, self.mms
        self.P = [interp_p2(cg.mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
        self.U = np.concatenate([interp_p2(cg.mc, mms, "u1", 0.0), interp_p2(cg.mc, mms, "u2", 0.0)])
        self.Pc = interp_p1(cg.mc, mms, "p", 0.0)
        self.P_old, self.U_old = [p.copy() for p in self.P], self.U.copy()
        fineP = [interp_p2(fg.mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
        fineU = np.concatenate([interp_p2(fg.mc, mms, "u1", 0.0), interp_p2(fg.mc, mms, "u2", 0.0)])
        ProlP = [prolong_p2(cg.mp, fg.mp, p) for p in self.P]
        ProlU = prolong_u(cg.mc, fg.mc, self.U)
        self.e = {}
        n2f = fg.mc.n2 ** 2
        for sd in self.subs:
            mesh = self._fine_mesh(sd.region)
            nodes, _, _ = sd.p2_nodes(mesh)
            cls = sd.classify_p2(mesh)
            if sd.region == POROUS:
                vals = [np.where(cls == 2, 0.0, fineP[i][nodes] - ProlP[i][nodes]) for i in range(3)]
            else:
                vals = [np.where(cls == 2, 0.0, fineU[c * n2f + nodes] - ProlU[c * n2f + nodes]) for c in range(2)]
                vals.append(np.zeros(len(sd.p1_nodes(mesh)[0])))
            self.e[sd.sid] = vals
        self.n = 0

    # -- Step 1 ----------------------------------------------------------------
    def coarse_step(self):
        t1 = self.t(self.n + 1)
        self.P_old, self.U_old = [p.copy() for p in self.P], self.U.copy()
        P_new = porous_step(self.cg, self.mms, self.P, self.U, t1)
        U_new, P_c, self.newton_its = ns_step(self.cg, self.mms, self.U, self.Pc, self.P[0], t1,
                                              convection=self.convection)
        self.P, self.U, self.Pc = P_new, U_new, P_c

    # -- Step 3 (1): local porous corrections, Eqs. (5.5)-(5.7) ----------------
    def _porous_ops(self, sd):
        key = ("p", sd.sid)
        if key not in self._cache:
            mesh = self.fg.mp
            E = mesh.elements_in_box(sd.x0, sd.x1, sd.y0, sd.y1)
            M, K = forms.p2_mass_stiff(mesh, E)
            G = forms.gamma_forms(mesh, sd.x0, sd.x1)[0] if sd.touches_gamma else None
            self._cache[key] = (E, M, K, G)
        return self._cache[key]

    def local_porous(self, sd, pro):
        co, mesh, mms = self.co, self.fg.mp, self.mms
        t1 = self.t(self.n + 1)
        E, M, K, G = self._porous_ops(sd)
        nodes, _, _ = sd.p2_nodes(mesh)
        cls = sd.classify_p2(mesh)
        nn = mesh.n2 ** 2
        PF1, Pf1, Pm1 = pro["P1"]
        PF0, Pf0, Pm0 = pro["P0"]
        Q = [forms.load_p2(mesh, E, lambda X, nm=nm: mms(nm, X, t1)) for nm in ("qF", "qf", "qm")]

        def full(loc):           # local lattice vector -> region vector (0 elsewhere)
            v = np.zeros(nn)
            v[nodes] = loc
            return v
        eF, ef, em = [full(v) for v in self.e[sd.sid]]
        gam = np.zeros(nn)
        if G is not None:
            n2c = self.fg.mc.n2 ** 2
            gam = -G @ (self.fg.T_cp @ pro["U0"][n2c:])     # + <u_cH^n . n_c, v_F>_Gamma
        # coarse-residual bracket of (5.5)-(5.7) plus the lagged e^n terms
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
        xy = mesh.p2_coords()[nodes]
        out = []
        for i, nm in enumerate(("pF", "pf", "pm")):
            dvals = np.where(cls == 1, mms(nm, xy, t1) - pro["P1"][i][nodes], 0.0)
            Al = A[i][nodes][:, nodes]
            out.append(_solve_dirichlet(Al.tocsr(), rhs[i][nodes], cls != 0, dvals))
        return out

    # -- Step 3 (2): local conduit (Oseen) correction, Eq. (5.8) ----------------
    def local_conduit(self, sd, pro):
        co, mesh, mms = self.co, self.fg.mc, self.mms
        t1 = self.t(self.n + 1)
        E = mesh.elements_in_box(sd.x0, sd.x1, sd.y0, sd.y1)
        Mv, S, Bq = forms.stokes_blocks(mesh, E)
        n2, n1 = mesh.n2 ** 2, mesh.n1 ** 2
        W1, W0, Pp = pro["U1"], pro["U0"], pro["Pc1"]
        if self.convection:
            cv, Nm = forms.convection(mesh, E, W1)
        else:
            cv, Nm = np.zeros(2 * n2), sps.csr_matrix((2 * n2, 2 * n2))
        if sd.touches_gamma:
            G, Gx = forms.gamma_forms(mesh, sd.x0, sd.x1)
            Gblk = sps.block_diag([G, sps.csr_matrix((n2, n2))]).tocsr()
            gam = conduit_gamma_rhs(self.fg, pro["P0"][0], co, mesh, G, Gx)
        else:
            Gblk = sps.csr_matrix((2 * n2, 2 * n2))
            gam = np.zeros(2 * n2)
        F = np.concatenate([forms.load_p2(mesh, E, lambda X: mms("f1", X, t1)),
                            forms.load_p2(mesh, E, lambda X: mms("f2", X, t1))])
        Avis = co.nu * co.eta * S + co.eta * co.beta * Gblk        # a_{c,eta}
        A = (co.eta / co.dt) * Mv + Avis + co.eta * Nm
        nodes, _, _ = sd.p2_nodes(mesh)
        pn, I, J = sd.p1_nodes(mesh)
        cls = sd.classify_p2(mesh)
        pfix = sd.artificial_p1(I, J)
        en = np.zeros(2 * n2)
        en[nodes], en[n2 + nodes] = self.e[sd.sid][0], self.e[sd.sid][1]
        # right-hand side of (5.8): source minus the coarse bracket, Gamma terms, lagged e^n
        rv = co.eta * F - ((co.eta / co.dt) * (Mv @ (W1 - W0)) + Avis @ W1
                           - co.eta * (Bq.T @ Pp) + co.eta * cv) + gam + (co.eta / co.dt) * (Mv @ en)
        rq = -co.eta * (Bq @ W1)
        vi = np.concatenate([nodes, n2 + nodes])
        K = sps.bmat([[A[vi][:, vi], -co.eta * Bq.T[vi][:, pn]],
                      [co.eta * Bq[pn][:, vi], None]]).tocsr()
        rhs = np.concatenate([rv[vi], rq[pn]])
        xy = mesh.p2_coords()[nodes]
        dv = [np.where(cls == 1, mms(nm, xy, t1) - W1[c * n2 + nodes], 0.0)
              for c, nm in enumerate(("u1", "u2"))]
        dmask = np.concatenate([cls != 0, cls != 0, pfix])
        dvals = np.concatenate([dv[0], dv[1], np.zeros(len(pn))])
        z = _solve_dirichlet(K, rhs, dmask, dvals)
        nv = len(nodes)
        return [z[:nv], z[nv:2 * nv], z[2 * nv:]]

    # -- Steps 3 and 4 -------------------------------------------------------------
    def prolonged(self):
        cg, fg = self.cg, self.fg
        return dict(
            P1=[prolong_p2(cg.mp, fg.mp, p) for p in self.P],
            P0=[prolong_p2(cg.mp, fg.mp, p) for p in self.P_old],
            U1=prolong_u(cg.mc, fg.mc, self.U),
            U0=prolong_u(cg.mc, fg.mc, self.U_old),
            Pc1=prolong_p1(cg.mc, fg.mc, self.Pc))

    def local_step(self):
        pro = self.prolonged()
        enew = {}
        for sd in self.subs:
            if sd.region == POROUS:
                enew[sd.sid] = self.local_porous(sd, pro)
            else:
                enew[sd.sid] = self.local_conduit(sd, pro)
        self.e = enew
        self.n += 1
        self._pro = pro
        if self.previous == "merged":
            # reading R18: the next step lags the merged correction
            f = self.merged()
            n2 = self.fg.mc.n2 ** 2
            for sd in self.subs:
                mesh = self._fine_mesh(sd.region)
                nodes, _, _ = sd.p2_nodes(mesh)
                cls = sd.classify_p2(mesh)
                if sd.region == POROUS:
                    self.e[sd.sid] = [np.where(cls == 2, 0.0, (f[k] - pro["P1"][i])[nodes])
                                      for i, k in enumerate(("pF", "pf", "pm"))]
                else:
                    d = f["u"] - pro["U1"]
                    self.e[sd.sid] = [np.where(cls == 2, 0.0, d[c * n2 + nodes]) for c in range(2)] + \
                                     [self.e[sd.sid][2]]
        return pro

    def merged(self):
        """Step 4 with partition-of-unity weights (reading R4): fine fields
        u (component-blocked), p (P1), pF, pf, pm on the region lattices."""
        pro = self._pro
        fg = self.fg
        out = {}
        for region in (POROUS, CONDUIT):
            mesh = self._fine_mesh(region)
            a = np.arange(mesh.n2)
            wx = 1.0 / owner_counts(self.cuts[(region, 0)], a)
            wy = 1.0 / owner_counts(self.cuts[(region, 1)], a)
            i1 = np.arange(mesh.n1)
            vx = 1.0 / owner_counts(self.cuts[(region, 0)], 2 * i1)
            vy = 1.0 / owner_counts(self.cuts[(region, 1)], 2 * i1)
            n2 = mesh.n2 ** 2
            if region == POROUS:
                acc = [p.copy() for p in pro["P1"]]
            else:
                acc = [pro["U1"][:n2].copy(), pro["U1"][n2:].copy(), pro["Pc1"].copy()]
            for sd in self.subs:
                if sd.region != region:
                    continue
                dx0, dx1, dy0, dy1 = sd.d
                nodes, A, B = sd.p2_nodes(mesh)
                inD = (A >= 2 * dx0) & (A <= 2 * dx1) & (B >= 2 * dy0) & (B <= 2 * dy1)
                w = wx[A] * wy[B]
                nv = 3 if region == POROUS else 2
                for k in range(nv):
                    acc[k][nodes[inD]] += w[inD] * self.e[sd.sid][k][inD]
                if region == CONDUIT:
                    pn, I, J = sd.p1_nodes(mesh)
                    inDp = (I >= dx0) & (I <= dx1) & (J >= dy0) & (J <= dy1)
                    wp = vx[I] * vy[J]
                    acc[2][pn[inDp]] += wp[inDp] * self.e[sd.sid][2][inDp]
            if region == POROUS:
                out["pF"], out["pf"], out["pm"] = acc
            else:
                out["u"] = np.concatenate([acc[0], acc[1]])
                out["p"] = acc[2]
        return out

    def coarse(self):
        return dict(pF=self.P[0], pf=self.P[1], pm=self.P[2], u=self.U, p=self.Pc)


def algorithm1(N, prm, dt, nsteps, convection=True):
    """Algorithm 1 (partitioned time stepping, Section 3.3) on one grid of N
    cells per unit length; returns the final fields."""
    co = Coefs(prm, dt)
    mms = MMS(prm)
    gp = GridProblem(N, co)
    P = [interp_p2(gp.mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
    U = np.concatenate([interp_p2(gp.mc, mms, "u1", 0.0), interp_p2(gp.mc, mms, "u2", 0.0)])
    Pc = interp_p1(gp.mc, mms, "p", 0.0)
    for n in range(nsteps):
        t1 = (n + 1) * dt
        Pn = porous_step(gp, mms, P, U, t1)
        U, Pc, _ = ns_step(gp, mms, U, Pc, P[0], t1, convection=convection)
        P = Pn
    return gp, dict(pF=P[0], pf=P[1], pm=P[2], u=U, p=Pc)
