"""Pins of the CPU oracle against what the paper and the mathematics fix
(no GPU).  Each test names the passage or fact it rests on."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sps
import sympy as sp

from oracle import forms
from oracle.fe import triangle_rule, p2_basis, p1_basis, gauss_legendre_01
from oracle.mesh import RegionMesh, POROUS, CONDUIT, make_subdomains, uniform_cuts, owner_counts
from oracle.mms import exact_ex1, sources, MMS, x, y, t
from oracle.norms import fe_errors
from oracle.scheme import (Oracle2D, algorithm1, Coefs, GridProblem, prolong_p2, prolong_u,
                           prolong_p1, interp_p2, interp_p1, _solve_dirichlet, conduit_gamma_rhs)

UNIT = dict(phi=[1.0] * 3, C=[1.0] * 3, k=[1.0] * 3, mu_tilde=1.0, sigma=1.0, sigma_star=1.0,
            rho=1.0, alpha=1.0, eta=1.0, nu=1.0)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ucuts(N, n):
    return {(r, a): uniform_cuts(N, n) for r in (POROUS, CONDUIT) for a in (0, 1)}


# --------------------------------------------------------------------------
# P3: quadrature and reference-element integrals
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", [3, 4, 6])
def test_triangle_rule_monomials(m):
    """int_T xi^a eta^b = a! b! / (a+b+2)! on the reference triangle, exact
    for a + b <= 2m - 2 (collapsed Gauss-Legendre)."""
    pts, w = triangle_rule(m)
    for a in range(2 * m - 1):
        for b in range(2 * m - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(got - exact) < 1e-14, (a, b)


def test_p2_reference_integrals():
    """P2 on a triangle: vertex functions integrate to 0, edge functions to
    |T|/3; the basis is a partition of unity and interpolates its nodes."""
    pts, w = triangle_rule(4)
    val, grad = p2_basis(pts)
    ints = w @ val
    assert np.allclose(ints[:3], 0.0, atol=1e-15)
    assert np.allclose(ints[3:], 0.5 / 3, atol=1e-15)
    assert np.allclose(val.sum(1), 1.0)
    assert np.allclose(grad.sum(1), 0.0, atol=1e-14)
    nodes = np.array([[0, 0], [1, 0], [0, 1], [.5, 0], [.5, .5], [0, .5]], float)
    v, _ = p2_basis(nodes)
    assert np.allclose(v, np.eye(6), atol=1e-15)


@pytest.mark.parametrize("N", [2, 5])
def test_assembled_forms_closed_forms(N):
    """Mass sums to the area, stiffness kills constants, strain kills rigid
    motions, the divergence form kills divergence-free fields and integrates
    div (x, 0) = 1 to the area, Gamma mass sums to |Gamma| = 1."""
    mp, mc = RegionMesh(N, POROUS), RegionMesh(N, CONDUIT)
    E = np.arange(2 * N * N)
    M, K = forms.p2_mass_stiff(mp, E)
    assert abs(M.sum() - 1.0) < 1e-13
    assert abs(K @ np.ones(K.shape[0])).max() < 1e-12
    Mv, S, Bq = forms.stokes_blocks(mc, E)
    xy = mc.p2_coords()
    n2 = mc.n2 ** 2
    rot = np.concatenate([-xy[:, 1], xy[:, 0]])
    assert abs(S @ rot).max() < 1e-12
    assert abs(Bq @ np.concatenate([xy[:, 0], -xy[:, 1]])).max() < 1e-13
    assert abs((Bq @ np.concatenate([xy[:, 0], 0 * xy[:, 0]])).sum() - 1.0) < 1e-13
    G, Gx = forms.gamma_forms(mc)
    assert abs(G.sum() - 1.0) < 1e-13
    # d_x of x along Gamma is 1: sum_a Gx[a, :] x = int_Gamma 1
    assert abs((Gx @ xy[:, 0]).sum() - 1.0) < 1e-13
    assert abs(forms.p1_mass(mc, E).sum() - 1.0) < 1e-13


def test_convection_newton_identity():
    """N(w) w = 2 c(w) and N(w) is the derivative of c (b_N is quadratic)."""
    mc = RegionMesh(3, CONDUIT)
    E = np.arange(18)
    rng = np.random.default_rng(1)
    w = rng.standard_normal(2 * mc.n2 ** 2)
    d = rng.standard_normal(w.size)
    c, Nm = forms.convection(mc, E, w)
    assert abs(Nm @ w - 2 * c).max() < 1e-13
    c2, _ = forms.convection(mc, E, w + d)
    cd, _ = forms.convection(mc, E, d)
    assert abs(c2 - c - Nm @ d - cd).max() < 1e-12


# --------------------------------------------------------------------------
# P1 / P2: counts and partition
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,nsub,ov", [(16, 4, 2), (64, 8, 4), (12, 3, 3)])
def test_counts_closed_form(N, nsub, ov):
    """(2N+1)^2 P2 and (N+1)^2 P1 nodes, 2N^2 triangles per region; free P2
    nodes of a box = product over axes of (2c - 1 + [face natural])."""
    m = RegionMesh(N, POROUS)
    assert m.el_p2.shape == (2 * N * N, 6)
    assert len(np.unique(m.el_p2)) == (2 * N + 1) ** 2
    assert len(np.unique(m.el_p1)) == (N + 1) ** 2
    mc = RegionMesh(N, CONDUIT)
    for sd in make_subdomains(N, ucuts(N, nsub), ov):
        mesh = m if sd.region == POROUS else mc
        cls = sd.classify_p2(mesh)
        cx, cy = sd.x1 - sd.x0, sd.y1 - sd.y0
        nat = 1 if sd.touches_gamma else 0
        assert (cls == 0).sum() == (2 * cx - 1) * (2 * cy - 1 + nat)
        _, I, J = sd.p1_nodes(mesh)
        nfix = sd.artificial_p1(I, J).sum()
        nart_x = (sd.x0 > 0) + (sd.x1 < N)
        nart_y = (sd.y0 > 0) + (sd.y1 < N)
        assert (cx + 1) * (cy + 1) - nfix == (cx + 1 - nart_x) * (cy + 1 - nart_y)


def _read_golden_partition():
    rows = []
    with open(os.path.join(GOLDEN, "ex1_partition_2d.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            left, right = line.split("|")
            lt = left.split()
            rows.append((lt[0], tuple(Fraction(v) for v in lt[1:]),
                         tuple(Fraction(v) for v in right.split())))
    return rows


@pytest.mark.parametrize("N", [4, 8, 16])
def test_partition_reproduces_example1(N):
    """Algorithm 3 Step 2 with 2 x 2 cores per region enlarged by 1/4
    reproduces the D and Omega boxes printed for Example 1 (Section 6)."""
    subs = make_subdomains(N, ucuts(N, 2), N // 4)
    got = set()
    for sd in subs:
        off = 0 if sd.region == POROUS else 1
        name = "porous" if sd.region == POROUS else "conduit"
        f = lambda v: Fraction(v, N)
        dx0, dx1, dy0, dy1 = sd.d
        got.add((name, (f(dx0), f(dx1), f(dy0) + off, f(dy1) + off),
                 (f(sd.x0), f(sd.x1), f(sd.y0) + off, f(sd.y1) + off)))
    want = set(_read_golden_partition())
    assert got == want


def test_pu_weights_sum_to_one():
    """Partition-of-unity weights over the closed cores sum to one at every node."""
    N = 24
    cuts = [0, 5, 13, 19, 24]
    a = np.arange(2 * N + 1)
    w = 1.0 / owner_counts(cuts, a)
    tot = np.zeros(len(a))
    c2 = np.array(cuts) * 2
    for k in range(len(cuts) - 1):
        tot += np.where((a >= c2[k]) & (a <= c2[k + 1]), w, 0.0)
    assert np.allclose(tot, 1.0)


# --------------------------------------------------------------------------
# P4: manufactured solution of Example 1
# --------------------------------------------------------------------------
def test_mms_interface_conditions_unit_parameters():
    """Example 1's exact solution satisfies div u = 0 and the five interface
    conditions of Section 2 on y = 1 when all parameters are 1."""
    ex = exact_ex1()
    u1, u2, p, pF, pf, pm = ex["u1"], ex["u2"], ex["p"], ex["pF"], ex["pf"], ex["pm"]
    assert sp.simplify(sp.diff(u1, x) + sp.diff(u2, y)) == 0
    on = {y: 1}
    # no flux for p_m and p_f
    assert sp.simplify(sp.diff(pm, y).subs(on)) == 0
    assert sp.simplify(sp.diff(pf, y).subs(on)) == 0
    # mass: u.n_c = k_F/mu grad p_F . n_p with n_c = (0,-1), n_p = (0,1)
    assert sp.simplify((-u2 - sp.diff(pF, y)).subs(on)) == 0
    # normal stress: -n_c.T n_c = p_F / rho, T_yy = 2 nu d_y u2 - p
    assert sp.simplify((-(2 * sp.diff(u2, y) - p) - pF).subs(on)) == 0
    # Beavers-Joseph: -P_tau(T n_c) = alpha nu / sqrt(k_F) P_tau(u + k_F/mu grad p_F)
    Txy = sp.diff(u1, y) + sp.diff(u2, x)
    assert sp.simplify((Txy - (u1 + sp.diff(pF, x))).subs(on)) == 0


def test_mms_sources_vs_finite_differences():
    """Sources derived symbolically match the strong form evaluated by
    central differences of the exact solution (non-unit parameters)."""
    prm = dict(UNIT, k=[0.3, 0.05, 0.002], sigma=2.0, sigma_star=0.7, nu=0.01, mu_tilde=1.3,
               phi=[0.5, 1.0, 2.0])
    mms = MMS(prm)
    rng = np.random.default_rng(2)
    P = rng.uniform(0.1, 0.9, (6, 2))
    tt = 0.37
    hs = 1e-4
    mu = prm["mu_tilde"]
    kF, kf, km = prm["k"]
    sst, s = prm["sigma_star"] * kf / mu, prm["sigma"] * km / mu
    F = lambda nm, X, T: mms(nm, X, T)

    def lap(nm, X):
        ex_, ey_ = np.array([hs, 0]), np.array([0, hs])
        return (F(nm, X + ex_, tt) + F(nm, X - ex_, tt) + F(nm, X + ey_, tt) + F(nm, X - ey_, tt)
                - 4 * F(nm, X, tt)) / hs ** 2

    def dt_(nm, X):
        return (F(nm, X, tt + hs) - F(nm, X, tt - hs)) / (2 * hs)
    qF = 0.5 * dt_("pF", P) - kF / mu * lap("pF", P) + sst * (F("pF", P, tt) - F("pf", P, tt))
    assert np.allclose(qF, mms("qF", P, tt), atol=1e-5)
    qm = 2.0 * dt_("pm", P) - km / mu * lap("pm", P) + s * (F("pm", P, tt) - F("pf", P, tt))
    assert np.allclose(qm, mms("qm", P, tt), atol=1e-5)
    qf = 1.0 * dt_("pf", P) - kf / mu * lap("pf", P) + sst * (F("pf", P, tt) - F("pF", P, tt)) \
        + s * (F("pf", P, tt) - F("pm", P, tt))
    assert np.allclose(qf, mms("qf", P, tt), atol=1e-5)
    Pc = P + np.array([0.0, 1.0])
    # f_1 = du1/dt - nu lap u1 + dp/dx + u . grad u1   (div u = 0)
    ex_, ey_ = np.array([hs, 0]), np.array([0, hs])
    dx = lambda nm: (F(nm, Pc + ex_, tt) - F(nm, Pc - ex_, tt)) / (2 * hs)
    dy = lambda nm: (F(nm, Pc + ey_, tt) - F(nm, Pc - ey_, tt)) / (2 * hs)
    f1 = (dt_("u1", Pc) - prm["nu"] * lap("u1", Pc) + dx("p")
          + F("u1", Pc, tt) * dx("u1") + F("u2", Pc, tt) * dy("u1"))
    assert np.allclose(f1, mms("f1", Pc, tt), atol=1e-5)
    # f_2 = du2/dt - nu lap u2 + dp/dy + u . grad u2
    f2 = (dt_("u2", Pc) - prm["nu"] * lap("u2", Pc) + dy("p")
          + F("u1", Pc, tt) * dx("u2") + F("u2", Pc, tt) * dy("u2"))
    assert np.allclose(f2, mms("f2", Pc, tt), atol=1e-5)


# --------------------------------------------------------------------------
# Scheme-level pins
# --------------------------------------------------------------------------
def test_algorithm1_rates_p2():
    """Algorithm 1 with P2-P1 + P2 at small dt: L2 errors fall like h^3 for the
    P2 fields and h^2 for the P1 pressure; H1 errors like h^2 (Theorem 3.3 in
    the paper's notation with r + 1 = 2 gives at least these orders)."""
    T, dt = 0.004, 1e-3
    ex = exact_ex1()
    mmsx = MMS(UNIT)
    errs = []
    for N in (4, 8, 16):
        gp, f = algorithm1(N, UNIT, dt, int(round(T / dt)))

        def exact(name):
            fn = sp.lambdify((x, y), ex[name].subs(t, T), "numpy")
            gx = sp.lambdify((x, y), sp.diff(ex[name], x).subs(t, T), "numpy")
            gy = sp.lambdify((x, y), sp.diff(ex[name], y).subs(t, T), "numpy")
            bc = lambda v, X: np.broadcast_to(np.asarray(v, float), (X.shape[0],))
            return lambda X: (bc(fn(X[:, 0], X[:, 1]), X),
                              np.stack([bc(gx(X[:, 0], X[:, 1]), X), bc(gy(X[:, 0], X[:, 1]), X)], 1))
        n2 = gp.mc.n2 ** 2
        row = []
        for nm in ("pF", "pf", "pm"):
            row += list(fe_errors(gp.mp, f[nm], exact(nm)))
        row += list(fe_errors(gp.mc, f["u"][:n2], exact("u1")))
        row += list(fe_errors(gp.mc, f["u"][n2:], exact("u2")))
        row.append(fe_errors(gp.mc, f["p"], exact("p"), degree=1)[0])
        errs.append(row)
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    # P2 fields pF, pf, pm, u1, u2: (L2, H1) at columns (0,1) (2,3) (4,5) (6,7) (8,9)
    l2, h1 = rates[:, 0:10:2], rates[:, 1:10:2]
    # finest pair at the asymptotic rates; p_m, the steepest field, is
    # pre-asymptotic on the coarsest grid
    assert (l2[-1] > 2.7).all() and (h1[-1] > 1.8).all(), rates
    assert (l2 > 2.4).all() and (h1 > 1.6).all(), rates
    assert (rates[:, 10] > 1.8).all(), rates


def test_h_equals_H_gives_zero_corrections():
    """H = h: the coarse solution already solves the fine residual equations,
    so every local correction vanishes and the merged field equals
    Algorithm 1 on that grid (Algorithm 3 Steps 3-4 with T_h = T_H)."""
    o = Oracle2D(8, 8, ucuts(8, 4), 1, UNIT, 0.05)
    o.init()
    for _ in range(2):
        o.coarse_step()
        o.local_step()
    emax = max(abs(v).max() for vs in o.e.values() for v in vs)
    assert emax < 1e-11
    _, f = algorithm1(8, UNIT, 0.05, 2)
    m = o.merged()
    for k in f:
        assert abs(m[k] - f[k]).max() < 1e-11, k


def _bf2_run(NH, Nh, prm, dt, nsteps):
    """One subdomain per region: merged result vs an independently written
    global fine solve.  Porous: Algorithm 1 Step 1 on T_h fed by the
    prolonged coarse u_cH^n on Gamma; conduit: the Oseen problem linearised
    about the prolonged u_cH^{n+1}, i.e. one Newton step for the fine
    Navier-Stokes equations with the coarse p_FH^n on Gamma."""
    cuts = {(r, a): [0, Nh] for r in (POROUS, CONDUIT) for a in (0, 1)}
    o = Oracle2D(NH, Nh, cuts, 0, prm, dt)
    o.init()
    mms = o.mms
    fg, co = o.fg, o.co
    mp, mc = fg.mp, fg.mc
    n2 = mc.n2 ** 2
    E = np.arange(2 * Nh * Nh)
    xp, xc = mp.p2_coords(), mc.p2_coords()
    X = [interp_p2(mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
    u = np.concatenate([interp_p2(mc, mms, "u1", 0.0), interp_p2(mc, mms, "u2", 0.0)])
    Gblk = sps.block_diag([fg.Gc, sps.csr_matrix((n2, n2))]).tocsr()
    worst = 0.0
    for n in range(nsteps):
        t1 = (n + 1) * dt
        o.coarse_step()
        o.local_step()
        pro = o._pro
        M, K = fg.M, fg.K
        Q = [forms.load_p2(mp, E, lambda Y, nm=nm: mms(nm, Y, t1)) for nm in ("qF", "qf", "qm")]
        gam = -fg.Gp @ (fg.T_cp @ pro["U0"][n2:])
        A = [(co.tau[0] + co.sst) * M + co.kap[0] * K, (co.tau[1] + co.s + co.sst) * M + co.kap[1] * K,
             (co.tau[2] + co.s) * M + co.kap[2] * K]
        rhs = [Q[0] + co.tau[0] * (M @ X[0]) + co.sst * (M @ X[1]) + gam,
               Q[1] + co.tau[1] * (M @ X[1]) + co.s * (M @ X[2]) + co.sst * (M @ X[0]),
               Q[2] + co.tau[2] * (M @ X[2]) + co.s * (M @ X[1])]
        X = [_solve_dirichlet(A[i], rhs[i], fg.dir_p, mms(nm, xp, t1))
             for i, nm in enumerate(("pF", "pf", "pm"))]
        W = pro["U1"]
        cv, Nm = forms.convection(mc, E, W)
        F = np.concatenate([forms.load_p2(mc, E, lambda Y: mms("f1", Y, t1)),
                            forms.load_p2(mc, E, lambda Y: mms("f2", Y, t1))])
        Aop = (co.eta / co.dt) * fg.Mv + co.nu * co.eta * fg.S + co.eta * co.beta * Gblk + co.eta * Nm
        J = sps.bmat([[Aop, -co.eta * fg.Bq.T], [co.eta * fg.Bq, None]]).tocsr()
        rv = co.eta * F + (co.eta / co.dt) * (fg.Mv @ u) + co.eta * cv \
            + conduit_gamma_rhs(fg, pro["P0"][0], co)
        rq = np.zeros(fg.Bq.shape[0])
        g = np.concatenate([mms("u1", xc, t1), mms("u2", xc, t1), np.zeros(len(rq))])
        dm = np.concatenate([fg.dir_c, fg.dir_c, np.zeros(len(rq), bool)])
        z = _solve_dirichlet(J, np.concatenate([rv, rq]), dm, g)
        u, p = z[:2 * n2], z[2 * n2:]
        m = o.merged()
        ref = dict(pF=X[0], pf=X[1], pm=X[2], u=u, p=p)
        for k in ref:
            worst = max(worst, abs(m[k] - ref[k]).max() / max(1.0, abs(ref[k]).max()))
    return worst


def test_single_subdomain_equals_global_fine_solve():
    """BF2: with Omega_j = the whole region the local step is algebraically
    the global fine problem described above (substitute e = x_h - Pi_h x_H)."""
    prm = dict(UNIT, nu=0.1, k=[0.5, 0.2, 0.01], sigma=3.0)
    assert _bf2_run(2, 8, prm, 0.05, 3) < 1e-12


def test_local_incompressibility_and_symmetry():
    """P8: B_j (Pi_h u_cH^{n+1} + e_j) = 0 against every free local pressure
    test function.  P10: local porous matrices are symmetric positive
    definite."""
    prm = dict(UNIT, nu=0.05)
    o = Oracle2D(4, 16, ucuts(16, 4), 2, prm, 0.02)
    o.init()
    o.coarse_step()
    o.local_step()
    mesh = o.fg.mc
    n2 = mesh.n2 ** 2
    W1 = o._pro["U1"]
    for sd in o.subs:
        if sd.region == POROUS:
            E, M, K, _ = o._porous_ops(sd)
            nodes, _, _ = sd.p2_nodes(o.fg.mp)
            free = nodes[sd.classify_p2(o.fg.mp) == 0]
            A = (0.3 * M + 0.7 * K)[free][:, free].toarray()
            assert abs(A - A.T).max() < 1e-15 * max(1, abs(A).max())
            np.linalg.cholesky(A)
            continue
        E = mesh.elements_in_box(sd.x0, sd.x1, sd.y0, sd.y1)
        _, _, Bq = forms.stokes_blocks(mesh, E)
        nodes, _, _ = sd.p2_nodes(mesh)
        pn, I, J = sd.p1_nodes(mesh)
        u = W1.copy()
        u[nodes] += o.e[sd.sid][0]
        u[n2 + nodes] += o.e[sd.sid][1]
        div = (Bq @ u)[pn][~sd.artificial_p1(I, J)]
        assert abs(div).max() < 1e-12


def test_prolongation_is_exact_on_nested_grids():
    """Pi_h reproduces a coarse P2 / P1 function exactly: a quadratic
    (linear) polynomial interpolated on T_H and prolonged equals its fine
    interpolant."""
    for region in (POROUS, CONDUIT):
        c, f = RegionMesh(3, region), RegionMesh(12, region)
        q = lambda X: 1 + 2 * X[:, 0] - X[:, 1] + 3 * X[:, 0] * X[:, 1] - X[:, 1] ** 2 + 0.5 * X[:, 0] ** 2
        assert abs(prolong_p2(c, f, q(c.p2_coords())) - q(f.p2_coords())).max() < 1e-13
        l = lambda X: 1 + 2 * X[:, 0] - 3 * X[:, 1]
        assert abs(prolong_p1(c, f, l(c.p1_coords())) - l(f.p1_coords())).max() < 1e-13
