"""Pins of the 3D oracle (Kuhn tetrahedra, P2-P1 + P2, Example 2 of Section 6)
against what the paper and the mathematics fix (no GPU).  Each test names
the passage or fact it rests on."""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

from oracle import forms3
from oracle.fe3 import tet_rule, p1_basis3, p2_basis3, EDGES
from oracle.mesh3 import RegionMesh3, POROUS, CONDUIT, extend_core
from oracle.mms3 import exact_ex2_paper, exact_ex2, example2_params, MMS3, x, y, z, t
from oracle.scheme import _solve_dirichlet
from oracle.scheme3 import algorithm1_3d, region_dirichlet_p2_3d, prolong_p2_3d, prolong_p1_3d, _locate3

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# reference element (Section 3.2 with d = 3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", [2, 3, 5, 6])
def test_tet_rule_monomials(m):
    """int xi^a eta^b zeta^c over the reference tetrahedron equals
    a! b! c! / (a+b+c+3)!, exactly for a + b + c <= 2m - 3."""
    pts, w = tet_rule(m)
    deg = 2 * m - 3
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
                got = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
                assert abs(got - exact) < 1e-15, (m, a, b, c)


def test_p2_tet_basis():
    """The ten P2 functions interpolate their nodes (vertices, then the
    midpoints of the edges in the stated order), sum to one, integrate to
    -|T|/20 (vertices) and |T|/5 (edges), and their gradients match finite
    differences."""
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    nodes = np.vstack([verts] + [0.5 * (verts[i] + verts[j]) for i, j in EDGES])
    val, _ = p2_basis3(nodes)
    assert np.allclose(val, np.eye(10), atol=1e-15)
    pts, w = tet_rule(4)
    val, grad = p2_basis3(pts)
    assert np.allclose(val.sum(1), 1.0)
    ints = w @ val
    assert np.allclose(ints[:4], -1.0 / 6 / 20, atol=1e-15)
    assert np.allclose(ints[4:], 1.0 / 6 / 5, atol=1e-15)
    rng = np.random.default_rng(0)
    p = rng.dirichlet(np.ones(4), 20)[:, 1:]
    eps = 1e-6
    _, g = p2_basis3(p)
    for k in range(3):
        d = np.zeros(3)
        d[k] = eps
        fd = (p2_basis3(p + d)[0] - p2_basis3(p - d)[0]) / (2 * eps)
        assert np.allclose(g[:, :, k], fd, atol=1e-8)
    lam, dl = p1_basis3(p)
    assert np.allclose(lam.sum(1), 1.0) and np.allclose(dl.sum(0), 0.0)


# --------------------------------------------------------------------------
# meshes (P1 counts; conformity and nesting of the Kuhn split)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", [1, 3])
def test_kuhn_mesh_conforming(N):
    """6 N^3 tetrahedra of volume h^3/6 fill the cube; every interior face is
    shared by exactly two tetrahedra and the 12 N^2 boundary triangles by one;
    each P2 edge node is the midpoint of its edge; (2N+1)^3 P2 and (N+1)^3 P1
    nodes, all used."""
    for region in (POROUS, CONDUIT):
        m = RegionMesh3(N, region)
        c1, c2 = m.p1_coords(), m.p2_coords()
        assert len(c2) == (2 * N + 1) ** 3 and len(c1) == (N + 1) ** 3
        assert len(np.unique(m.el_p2)) == len(c2) and len(np.unique(m.el_p1)) == len(c1)
        vol = 0.0
        faces = {}
        for e in range(6 * N ** 3):
            V = c1[m.el_p1[e]]
            J = (V[1:] - V[0]).T
            vol += abs(np.linalg.det(J)) / 6
            assert np.allclose(J, m.jacobian(m.el_orient[e]))
            assert np.allclose(c2[m.el_p2[e, :4]], V)
            for k, (i, j) in enumerate(EDGES):
                assert np.allclose(c2[m.el_p2[e, 4 + k]], 0.5 * (V[i] + V[j]))
            for f in itertools.combinations(m.el_p1[e], 3):
                key = tuple(sorted(f))
                faces[key] = faces.get(key, 0) + 1
        assert abs(vol - 1.0) < 1e-13
        counts = np.array(list(faces.values()))
        assert set(counts) <= {1, 2}
        assert (counts == 1).sum() == 12 * N * N


def test_kuhn_meshes_nest():
    """T_h refines T_H (Section 4): every fine tetrahedron of the N = 4 mesh
    lies inside one tetrahedron of the N = 2 mesh."""
    for region in (POROUS, CONDUIT):
        cm, fm = RegionMesh3(2, region), RegionMesh3(4, region)
        off = np.array([0.0, 0.0, fm.z0])
        V = fm.p1_coords()[fm.el_p1] - off                      # (ne, 4, 3)
        eid, _ = _locate3(cm, V.mean(1))
        cv = cm.p1_coords()[cm.el_p1[eid]] - off                  # (ne, 4, 3)
        for q in range(4):
            J = np.transpose(cv[:, 1:] - cv[:, :1], (0, 2, 1))
            ref = np.linalg.solve(J, (V[:, q] - cv[:, 0])[:, :, None])[:, :, 0]
            lam = np.concatenate([1 - ref.sum(1, keepdims=True), ref], 1)
            assert lam.min() > -1e-12


# --------------------------------------------------------------------------
# assembled forms: closed forms
# --------------------------------------------------------------------------
def test_forms3_closed_forms():
    """Mass and stiffness on the unit cube: int 1 = 1, int x^2 y z = 1/12,
    K 1 = 0, int |grad (x - 2y + 3z)|^2 = 14; strain: rigid motions in the
    kernel, int 2 D(u):D(u) = 2 for u = (x,0,0); divergence: B u = 3 int psi
    for u = (x, y, z); convection: N(w) w = 2 c(w), c(w) = M x for w = (x,0,0);
    Gamma: area 1 and int phi d_x x = int phi."""
    N = 2
    E = np.arange(6 * N ** 3)
    for region in (POROUS, CONDUIT):
        m = RegionMesh3(N, region)
        X = m.p2_coords()
        xx, yy, zz = X[:, 0], X[:, 1], X[:, 2] - m.z0
        M, K = forms3.p2_mass_stiff(m, E)
        one = np.ones(len(X))
        assert abs(one @ M @ one - 1.0) < 1e-13
        assert abs((xx ** 2) @ M @ (yy * zz) - 1.0 / 12) < 1e-13
        assert np.abs(K @ one).max() < 1e-12
        f = xx - 2 * yy + 3 * zz
        assert abs(f @ K @ f - 14.0) < 1e-12
        Mv, S, B = forms3.stokes_blocks(m, E)
        n2 = len(X)
        zero = np.zeros(n2)
        rigid = [np.concatenate(v) for v in ((one, zero, zero), (zero, one, zero), (zero, zero, one),
                                              (-yy, xx, zero), (zero, -zz, yy), (zz, zero, -xx))]
        for r in rigid:
            assert np.abs(S @ r).max() < 1e-12
        u = np.concatenate([xx, zero, zero])
        assert abs(u @ S @ u - 2.0) < 1e-12
        P1 = forms3.p1_mass(m, E)
        ones1 = np.ones(P1.shape[0])
        assert np.allclose(B @ np.concatenate([xx, yy, zz]), 3 * (P1 @ ones1), atol=1e-13)
        rng = np.random.default_rng(1)
        w = rng.standard_normal(3 * n2)
        cv, Nw = forms3.convection(m, E, w)
        assert np.allclose(Nw @ w, 2 * cv, atol=1e-11)
        cv, _ = forms3.convection(m, E, u)
        assert np.allclose(cv[:n2], M @ xx, atol=1e-13) and np.abs(cv[n2:]).max() < 1e-13
        G, Gx, Gy = forms3.gamma_forms(m)
        assert abs(one @ G @ one - 1.0) < 1e-13
        assert np.allclose(Gx @ xx, G @ one, atol=1e-13) and np.allclose(Gy @ yy, G @ one, atol=1e-13)
        assert np.abs(Gx @ yy).max() < 1e-13
    Gp = forms3.gamma_forms(RegionMesh3(N, POROUS))[0]
    Gc = forms3.gamma_forms(RegionMesh3(N, CONDUIT))[0]
    T = forms3.gamma_transfer(RegionMesh3(N, CONDUIT), RegionMesh3(N, POROUS))
    assert abs(Gp - T @ Gc @ T.T).max() < 1e-15


@pytest.mark.parametrize("N", [2, 3])
def test_p2_reproduces_quadratics(N):
    """P2 Galerkin reproduces a quadratic exactly: -lap u = -3 for
    u = x^2 + y z + z^2/2, all-Dirichlet, and with the Gamma face natural
    (flux du/dz = y + z through G)."""
    m = RegionMesh3(N, POROUS)
    E = np.arange(6 * N ** 3)
    _, K = forms3.p2_mass_stiff(m, E)
    X = m.p2_coords()
    ue = X[:, 0] ** 2 + X[:, 1] * X[:, 2] + 0.5 * X[:, 2] ** 2
    f = forms3.load_p2(m, E, lambda P: -3.0 + 0 * P[:, 0])
    L = m.n2
    q = np.arange(L ** 3)
    a, b, c = q % L, (q // L) % L, q // (L * L)
    alld = (a == 0) | (a == 2 * N) | (b == 0) | (b == 2 * N) | (c == 0) | (c == 2 * N)
    assert np.abs(_solve_dirichlet(K.tocsr(), f, alld, ue) - ue).max() < 1e-12
    G, _, _ = forms3.gamma_forms(m)
    d = region_dirichlet_p2_3d(m)
    assert not d[(c == 2 * N) & (a > 0) & (a < 2 * N) & (b > 0) & (b < 2 * N)].any()
    u2 = _solve_dirichlet(K.tocsr(), f + G @ (X[:, 1] + X[:, 2]), d, ue)
    assert np.abs(u2 - ue).max() < 1e-12


@pytest.mark.parametrize("region", [POROUS, CONDUIT])
def test_prolongation_exact_for_polynomials(region):
    """The prolongation between nested meshes evaluates the coarse element
    polynomial: exact for quadratics (P2) and linears (P1)."""
    cm, fm = RegionMesh3(2, region), RegionMesh3(6, region)
    q2 = lambda P: 1 + P[:, 0] - 2 * P[:, 1] + P[:, 2] ** 2 + P[:, 0] * P[:, 1] - 3 * P[:, 1] * P[:, 2]  # noqa: E731
    q1 = lambda P: 2 - P[:, 0] + 0.5 * P[:, 1] + 4 * P[:, 2]  # noqa: E731
    assert np.abs(prolong_p2_3d(cm, fm, q2(cm.p2_coords())) - q2(fm.p2_coords())).max() < 1e-13
    assert np.abs(prolong_p1_3d(cm, fm, q1(cm.p1_coords())) - q1(fm.p1_coords())).max() < 1e-13


# --------------------------------------------------------------------------
# Example 2's manufactured solution (Section 6) and the model (Section 2)
# --------------------------------------------------------------------------
def _interface_residuals(ex, zs, zg, sign):
    """Interface conditions of the model (Section 2) at the horizontal
    interface z = zg with n_c = (0, 0, sign) and all parameters 1:
    u . n_c = -grad p_F . n_c (mass), -n_c . T n_c = p_F (normal force),
    -P_tau(T n_c) = P_tau(u + grad p_F) (Beavers-Joseph with the Darcy
    velocity), T = 2 D(u) - p I; and div u = 0 in the conduit."""
    u = [ex["u1"], ex["u2"], ex["u3"]]
    X = [x, y, zs]
    pF, p = ex["pF"], ex["p"]
    n = [0, 0, sign]

    def Tn(i):
        return sum((sp.diff(u[i], X[j]) + sp.diff(u[j], X[i])) * n[j] for j in range(3)) - p * n[i]
    res = [sum(u[i] * n[i] for i in range(3)) + sum(sp.diff(pF, X[i]) * n[i] for i in range(3)),
           -sum(n[i] * Tn(i) for i in range(3)) - pF]
    for i in range(2):
        res.append(-Tn(i) - (u[i] + sp.diff(pF, X[i])))
    res = [r.subs(zs, zg) for r in res]
    res.append(sum(sp.diff(u[i], X[i]) for i in range(3)))
    return [sp.simplify(sp.expand(r)) for r in res]


def test_example2_interface_conditions_paper_coordinates():
    """Example 2's fields, as printed, satisfy the interface conditions at
    z = 0 (n_c = +e_z: the conduit lies below) and are divergence free."""
    zp = sp.Symbol("zp", real=True)
    assert _interface_residuals(exact_ex2_paper(zp), zp, 0, 1) == [0] * 5


def test_example2_reflection_keeps_the_conditions():
    """The reflected fields (porous region below z = 1, n_c = -e_z) satisfy
    the same conditions, and agree with the printed ones at mirrored points."""
    ex = exact_ex2()
    assert _interface_residuals(ex, z, 1, -1) == [0] * 5
    zp = sp.Symbol("zp", real=True)
    pe = exact_ex2_paper(zp)
    pt = {x: sp.Rational(3, 10), y: sp.Rational(7, 10), t: sp.Rational(1, 5)}
    for nm, sgn in (("pF", 1), ("pf", 1), ("pm", 1), ("u1", 1), ("u2", 1), ("u3", -1), ("p", 1)):
        a = ex[nm].subs({**pt, z: sp.Rational(13, 10)})
        b = sgn * pe[nm].subs({**pt, zp: sp.Rational(-3, 10)})
        assert abs(float(a - b)) < 1e-14, nm


def test_example2_sources_match_finite_differences():
    """The sources q_F, q_f, q_m and f = (f_1, f_2, f_3) equal the strong
    form (Section 2 equations with Example 2's parameters) applied to the
    exact fields by central differences, at random points of both regions."""
    prm = example2_params()
    mms = MMS3(prm)
    rng = np.random.default_rng(5)
    h = 1e-3

    def F(nm, P, tt):
        return mms(nm, P, tt)

    def d1(nm, P, tt, k):
        e = np.zeros(3)
        e[k] = h
        return (F(nm, P + e, tt) - F(nm, P - e, tt)) / (2 * h)

    def d2(nm, P, tt, k, l):
        ek, el = np.zeros(3), np.zeros(3)
        ek[k], el[l] = h, h
        return (F(nm, P + ek + el, tt) - F(nm, P + ek - el, tt) - F(nm, P - ek + el, tt)
                + F(nm, P - ek - el, tt)) / (4 * h * h)

    def dt(nm, P, tt):
        return (F(nm, P, tt + h) - F(nm, P, tt - h)) / (2 * h)

    kF, kf, km = prm["k"]
    Pp = rng.uniform(0.1, 0.9, (8, 3))
    Pc = Pp + np.array([0, 0, 1.0])
    tt = 0.37
    lap = lambda nm, P: sum(d2(nm, P, tt, k, k) for k in range(3))  # noqa: E731
    pF, pf, pm = (F(nm, Pp, tt) for nm in ("pF", "pf", "pm"))
    qF = dt("pF", Pp, tt) - kF * lap("pF", Pp) + kf * (pF - pf)
    qf = dt("pf", Pp, tt) - kf * lap("pf", Pp) + kf * (pf - pF) + km * (pf - pm)
    qm = dt("pm", Pp, tt) - km * lap("pm", Pp) + km * (pm - pf)
    for nm, v in (("qF", qF), ("qf", qf), ("qm", qm)):
        assert np.allclose(F(nm, Pp, tt), v, rtol=1e-5, atol=1e-5), nm
    U = [F("u%d" % (c + 1), Pc, tt) for c in range(3)]
    for c in range(3):
        un = "u%d" % (c + 1)
        visc = -sum(d2(un, Pc, tt, j, j) + d2("u%d" % (j + 1), Pc, tt, c, j) for j in range(3))
        conv = sum(U[j] * d1(un, Pc, tt, j) for j in range(3))
        f = dt(un, Pc, tt) + visc + d1("p", Pc, tt, c) + conv
        assert np.allclose(F("f%d" % (c + 1), Pc, tt), f, rtol=1e-5, atol=1e-5), c


# --------------------------------------------------------------------------
# Algorithm 3 Step 2: the printed 3D partition
# --------------------------------------------------------------------------
def _read_golden_3d():
    regions, rows = {}, []
    with open(os.path.join(GOLDEN, "ex2_partition_3d.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "REGION":
                regions[tok[1]] = tuple(Fraction(v) for v in tok[2:])
            else:
                d, o = line.split("|")
                d = d.split()
                rows.append((d[0], tuple(Fraction(v) for v in d[1:]), tuple(Fraction(v) for v in o.split())))
    return regions, rows


def test_example2_partition_boxes():
    """Section 6, Example 2: the sixteen printed boxes D_j tile their regions
    (2 x 2 x 2 each, disjoint, volumes adding up), and the printed Omega_j are
    the D_j extended on every side by half their extent along that axis,
    clipped to the region."""
    regions, rows = _read_golden_3d()
    assert len(rows) == 16
    for reg, box in regions.items():
        mine = [(d, o) for nm, d, o in rows if nm[0] == reg]
        assert len(mine) == 8
        vol = lambda b: (b[1] - b[0]) * (b[3] - b[2]) * (b[5] - b[4])  # noqa: E731
        assert sum(vol(d) for d, _ in mine) == vol(box)
        for (d1, _), (d2, _) in itertools.combinations(mine, 2):
            overlap = [max(0, min(d1[2 * k + 1], d2[2 * k + 1]) - max(d1[2 * k], d2[2 * k])) for k in range(3)]
            assert overlap[0] * overlap[1] * overlap[2] == 0
        for d, o in mine:
            assert all(box[2 * k] <= d[2 * k] < d[2 * k + 1] <= box[2 * k + 1] for k in range(3))
            assert extend_core(d, box) == o, (d, o)


# --------------------------------------------------------------------------
# Algorithm 1 (Section 3.3) in 3D: P2 rates
# --------------------------------------------------------------------------
def test_algorithm1_3d_rates():
    """Algorithm 1 with P2-P1 + P2 on the Kuhn meshes, Example 2's fields and
    parameters with k_m = 1 (the matrix pressure then resolves on these grids
    like the others), dt = 1e-3, one step: between N = 4 and N = 8 the L2
    errors of p_F, p_f, p_m and u fall at rate > 2.5 (P2: 3) and the H1
    errors at > 1.8 (P2: 2); the P1 pressure's L2 error at > 2."""
    prm = example2_params()
    prm["k"] = [1.0, 1.0, 1.0]
    mms = MMS3(prm)
    dt = 1e-3
    errs = []
    for N in (4, 8):
        gp, f = algorithm1_3d(N, prm, dt, 1)
        E = np.arange(6 * N ** 3)
        out = {}
        for nm in ("pF", "pf", "pm"):
            e = f[nm] - mms(nm, gp.mp.p2_coords(), dt)
            out[nm] = (np.sqrt(e @ gp.M @ e), np.sqrt(e @ gp.K @ e))
        Mc, Kc = forms3.p2_mass_stiff(gp.mc, E)
        n2 = gp.mc.n2 ** 3
        eu = [f["u"][c * n2:(c + 1) * n2] - mms("u%d" % (c + 1), gp.mc.p2_coords(), dt) for c in range(3)]
        out["u"] = (np.sqrt(sum(v @ Mc @ v for v in eu)), np.sqrt(sum(v @ Kc @ v for v in eu)))
        ep = f["p"] - mms("p", gp.mc.p1_coords(), dt)
        out["p"] = (np.sqrt(ep @ forms3.p1_mass(gp.mc, E) @ ep), None)
        errs.append(out)
    for nm in ("pF", "pf", "pm", "u"):
        r0 = np.log2(errs[0][nm][0] / errs[1][nm][0])
        r1 = np.log2(errs[0][nm][1] / errs[1][nm][1])
        assert r0 > 2.5 and r1 > 1.8, (nm, r0, r1, errs)
    assert np.log2(errs[0]["p"][0] / errs[1]["p"][0]) > 2.0, errs


# --------------------------------------------------------------------------
# Algorithm 3 in 3D (Steps 1-4 on the Kuhn meshes)
# --------------------------------------------------------------------------
def _cuts3(N, n):
    from oracle.mesh3 import uniform_cuts
    return {(r, a): uniform_cuts(N, n) for r in (POROUS, CONDUIT) for a in range(3)}


def test_algorithm3_3d_h_equals_H_gives_zero_corrections():
    """H = h: the coarse solution already solves the fine residual equations
    of Step 3, so every correction vanishes and the merged field is
    Algorithm 1 on that grid."""
    from oracle.scheme3 import Oracle3D
    prm = example2_params()
    o = Oracle3D(2, 2, _cuts3(2, 2), 1, prm, 0.05)
    o.init()
    for _ in range(2):
        o.coarse_step()
        o.local_step()
    assert max(np.abs(v).max() for vs in o.e.values() for v in vs) < 1e-11
    _, f = algorithm1_3d(2, prm, 0.05, 2)
    m = o.merged()
    for k in f:
        assert np.abs(m[k] - f[k]).max() < 1e-11, k


def test_algorithm3_3d_merge_reproduces_a_fine_field():
    """Step 4 in 3D: with every correction set to I_h x - Pi_h x_H on its
    box, the merged field is x at every fine P2 and P1 node (uneven cores, a
    different overlap per axis, seams and corners where up to 8 cores meet)."""
    from oracle.scheme3 import Oracle3D
    cuts = {(r, a): [0, 1, 4] for r in (POROUS, CONDUIT) for a in range(3)}
    o = Oracle3D(1, 4, cuts, (1, 0, 2), example2_params(), 0.05)
    o.init()
    o._pro = pro = o.prolonged()
    rng = np.random.default_rng(3)
    mp, mc = o.fg.mp, o.fg.mc
    n2 = mc.n2 ** 3
    X = {"pF": rng.standard_normal(n2), "pf": rng.standard_normal(n2), "pm": rng.standard_normal(n2),
         "u": rng.standard_normal(3 * n2), "p": rng.standard_normal(mc.n1 ** 3)}
    for sd in o.subs:
        if sd.region == POROUS:
            nodes = sd.p2_nodes(mp)[0]
            o.e[sd.sid] = [X[nm][nodes] - pro["P1"][i][nodes] for i, nm in enumerate(("pF", "pf", "pm"))]
        else:
            nodes, pn = sd.p2_nodes(mc)[0], sd.p1_nodes(mc)[0]
            o.e[sd.sid] = ([X["u"][c * n2 + nodes] - pro["U1"][c * n2 + nodes] for c in range(3)]
                           + [X["p"][pn] - pro["Pc1"][pn]])
    m = o.merged()
    for k in X:
        assert np.abs(m[k] - X[k]).max() < 1e-12, k


def test_algorithm3_3d_single_subdomain_equals_global_fine_solve():
    """One subdomain per region (BF2) in 3D: the merged result equals an
    independently written global fine solve: the porous step of Algorithm 1
    on T_h fed by the prolonged coarse u_cH^n on Gamma, and the Oseen problem
    linearised about the prolonged u_cH^{n+1} (one Newton step of the fine
    Navier-Stokes equations) with the coarse p_FH^n on Gamma."""
    import scipy.sparse as sps
    from oracle.scheme import _solve_dirichlet
    from oracle.scheme3 import Oracle3D, conduit_gamma_rhs3, interp
    NH, Nh, dt = 2, 4, 0.05
    prm = dict(example2_params(), nu=0.1, k=[0.5, 0.2, 0.01], sigma=3.0)
    cuts = {(r, a): [0, Nh] for r in (POROUS, CONDUIT) for a in range(3)}
    o = Oracle3D(NH, Nh, cuts, 0, prm, dt)
    o.init()
    mms, fg, co = o.mms, o.fg, o.co
    mp, mc = fg.mp, fg.mc
    n2 = mc.n2 ** 3
    E = np.arange(6 * Nh ** 3)
    xp, xc = mp.p2_coords(), mc.p2_coords()
    X = [interp(mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
    u = np.concatenate([interp(mc, mms, "u%d" % (c + 1), 0.0) for c in range(3)])
    Gblk = sps.block_diag([fg.Gc, fg.Gc, sps.csr_matrix((n2, n2))]).tocsr()
    for n in range(2):
        t1 = (n + 1) * dt
        o.coarse_step()
        o.local_step()
        pro = o._pro
        M, K = fg.M, fg.K
        Q = [forms3.load_p2(mp, E, lambda Y, nm=nm: mms(nm, Y, t1)) for nm in ("qF", "qf", "qm")]
        gam = -fg.Gp @ (fg.T_cp @ pro["U0"][2 * n2:])
        A = [(co.tau[0] + co.sst) * M + co.kap[0] * K, (co.tau[1] + co.s + co.sst) * M + co.kap[1] * K,
             (co.tau[2] + co.s) * M + co.kap[2] * K]
        rhs = [Q[0] + co.tau[0] * (M @ X[0]) + co.sst * (M @ X[1]) + gam,
               Q[1] + co.tau[1] * (M @ X[1]) + co.s * (M @ X[2]) + co.sst * (M @ X[0]),
               Q[2] + co.tau[2] * (M @ X[2]) + co.s * (M @ X[1])]
        X = [_solve_dirichlet(A[i], rhs[i], fg.dir_p, mms(nm, xp, t1)) for i, nm in enumerate(("pF", "pf", "pm"))]
        cv, Nm = forms3.convection(mc, E, pro["U1"])
        F = np.concatenate([forms3.load_p2(mc, E, lambda Y, c=c: mms("f%d" % (c + 1), Y, t1)) for c in range(3)])
        Aop = (co.eta / co.dt) * fg.Mv + co.nu * co.eta * fg.S + co.eta * co.beta * Gblk + co.eta * Nm
        J = sps.bmat([[Aop, -co.eta * fg.Bq.T], [co.eta * fg.Bq, None]]).tocsr()
        rv = co.eta * F + (co.eta / co.dt) * (fg.Mv @ u) + co.eta * cv + conduit_gamma_rhs3(fg, pro["P0"][0], co)
        rq = np.zeros(fg.Bq.shape[0])
        g = np.concatenate([mms("u%d" % (c + 1), xc, t1) for c in range(3)] + [np.zeros(len(rq))])
        dm = np.concatenate([fg.dir_c] * 3 + [np.zeros(len(rq), bool)])
        z = _solve_dirichlet(J, np.concatenate([rv, rq]), dm, g)
        u, p = z[:3 * n2], z[3 * n2:]
        m = o.merged()
        for k, ref in dict(pF=X[0], pf=X[1], pm=X[2], u=u, p=p).items():
            assert np.abs(m[k] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), (n, k)
