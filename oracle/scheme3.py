"""Algorithm 1 (Section 3.3, partitioned time stepping) in 3D, plain FP64 with
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
from .mesh3 import RegionMesh3, POROUS, CONDUIT, PERMS
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
