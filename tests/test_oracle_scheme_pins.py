"""Scheme-level pins of the CPU oracle (no GPU): properties of Algorithm 3 that
the paper and the mathematics fix, checked so that a plausible mistake in the
oracle (a wrong seam weight, a dropped or swapped exchange term, a wrong
lattice) fails at least one of them.  Each test names the passage it rests on.
"""
import numpy as np
import pytest
import scipy.sparse as sps
import sympy as sp

from oracle import forms
from oracle.mesh import RegionMesh, POROUS, CONDUIT, uniform_cuts
from oracle.mms import MMS, exact_ex1, x, y, t
from oracle.norms import fe_errors, mass_norm
from oracle.scheme import Oracle2D, GridProblem, Coefs, porous_step, interp_p2, algorithm1

UNIT = dict(phi=[1.0] * 3, C=[1.0] * 3, k=[1.0] * 3, mu_tilde=1.0, sigma=1.0, sigma_star=1.0,
            rho=1.0, alpha=1.0, eta=1.0, nu=1.0)
# non-unit parameters with every coefficient distinct, so that swapping any two
# of them changes the scheme
SKEW = dict(UNIT, k=[0.3, 0.05, 0.002], sigma=4.0, sigma_star=0.7, mu_tilde=1.3, phi=[0.5, 1.0, 2.0],
            C=[1.5, 0.8, 1.0])

_EX = exact_ex1()


def exact(name, T):
    """Exact field of Example 1 at time T: X -> (values, gradients)."""
    fn = sp.lambdify((x, y), _EX[name].subs(t, T), "numpy")
    gx = sp.lambdify((x, y), sp.diff(_EX[name], x).subs(t, T), "numpy")
    gy = sp.lambdify((x, y), sp.diff(_EX[name], y).subs(t, T), "numpy")
    bc = lambda v, X: np.broadcast_to(np.asarray(v, float), (X.shape[0],))
    return lambda X: (bc(fn(X[:, 0], X[:, 1]), X),
                      np.stack([bc(gx(X[:, 0], X[:, 1]), X), bc(gy(X[:, 0], X[:, 1]), X)], 1))


def ucuts(N, n):
    return {(r, a): uniform_cuts(N, n) for r in (POROUS, CONDUIT) for a in (0, 1)}


def rel_mass(mesh, a, b, degree=2, ncomp=1):
    n = len(a) // ncomp
    num = sum(mass_norm(mesh, a[i * n:(i + 1) * n] - b[i * n:(i + 1) * n], degree) ** 2 for i in range(ncomp))
    den = sum(mass_norm(mesh, b[i * n:(i + 1) * n], degree) ** 2 for i in range(ncomp))
    return np.sqrt(num / den)


# --------------------------------------------------------------------------
# Algorithm 3 Step 4: the partition-of-unity correction
# --------------------------------------------------------------------------
SHIFTED = {(POROUS, 0): [0, 5, 7, 12], (POROUS, 1): [0, 4, 9, 12],
           (CONDUIT, 0): [0, 3, 8, 12], (CONDUIT, 1): [0, 6, 10, 12]}


@pytest.mark.parametrize("cuts,overlap", [(SHIFTED, 0), (SHIFTED, 1), (SHIFTED, 3),
                                          ({k: uniform_cuts(12, 4) for k in SHIFTED}, 2)])
def test_merge_reproduces_a_fine_field(cuts, overlap):
    """Step 4 with the partition-of-unity weights (reading R4): if every
    subdomain's correction equals I_h x - Pi_h x_H on its own lattice, the
    merged field is x itself at every fine P2 and P1 node.  A seam node
    shared by k closed cores gets k contributions, each weighted 1/k, so a
    wrong weight or the P1 weights taken on the wrong lattice breaks this at
    seams and cross points (uneven cuts: seams at odd and even positions)."""
    NH, Nh = 3, 12
    o = Oracle2D(NH, Nh, cuts, overlap, UNIT, 0.1)
    o.init()
    o._pro = o.prolonged()
    pro = o._pro
    rng = np.random.default_rng(11)
    mp, mc = o.fg.mp, o.fg.mc
    n2 = mc.n2 ** 2
    X = {"pF": rng.standard_normal(n2), "pf": rng.standard_normal(n2), "pm": rng.standard_normal(n2),
         "u": rng.standard_normal(2 * n2), "p": rng.standard_normal(mc.n1 ** 2)}
    for sd in o.subs:
        if sd.region == POROUS:
            nodes, _, _ = sd.p2_nodes(mp)
            o.e[sd.sid] = [X[nm][nodes] - pro["P1"][i][nodes] for i, nm in enumerate(("pF", "pf", "pm"))]
        else:
            nodes, _, _ = sd.p2_nodes(mc)
            pn, _, _ = sd.p1_nodes(mc)
            o.e[sd.sid] = [X["u"][c * n2 + nodes] - pro["U1"][c * n2 + nodes] for c in range(2)]
            o.e[sd.sid].append(X["p"][pn] - pro["Pc1"][pn])
    m = o.merged()
    for k in X:
        assert np.abs(m[k] - X[k]).max() < 1e-12, k


# --------------------------------------------------------------------------
# Theorem 5.4 (Section 5.2): rates of Algorithm 3 with the paper's setting
# --------------------------------------------------------------------------
def _broken(o, name, T):
    """Broken errors (L2, H1) of Section 5.2: each subdomain's own function
    Pi_h x_H + e_j over the elements of its core D_j, summed in squares."""
    pro, fg = o._pro, o.fg
    l2 = h1 = 0.0
    for sd in o.subs:
        if name in ("pF", "pf", "pm"):
            if sd.region != POROUS:
                continue
            mesh, k = fg.mp, ("pF", "pf", "pm").index(name)
            base = pro["P1"][k].copy()
        else:
            if sd.region != CONDUIT:
                continue
            mesh, k = fg.mc, (0 if name == "u1" else 1)
            n2 = mesh.n2 ** 2
            base = pro["U1"][k * n2:(k + 1) * n2].copy()
        nodes, _, _ = sd.p2_nodes(mesh)
        base[nodes] += o.e[sd.sid][k]
        E = mesh.elements_in_box(*sd.d)
        a, b = fe_errors(mesh, base, exact(name, T), 2, E)
        l2 += a * a
        h1 += b * b
    return np.sqrt(l2), np.sqrt(h1)


def test_algorithm3_rates_theorem_5_4():
    """Example 1 with the partition of Section 6 (2 x 2 cores per region,
    Omega = core enlarged by 1/4), h = H^2 and dt = h^2, at (H, h) = (1/2, 1/4)
    and (1/4, 1/16), T = 1/16.  Theorem 5.4 (r = 1) bounds the broken H1 errors
    by dt + h^r + H^(r+1) = O(h) (rate >= 1 per refinement of h; 0.9 allows for
    pre-asymptotic noise) and the broken L2 errors of p_f and p_m by
    dt + h^(r+1) = O(h^2) (rate >= 1.8).  The merged P1 pressure, which the
    theorem does not bound, converges with the coarse pressure, O(H^2) = O(h)
    (rate >= 0.9): the local problems take their pressure level from p_H."""
    T = 1.0 / 16
    errs, perr = [], []
    for H in (2, 4):
        Nh = H * H
        dt = 1.0 / Nh ** 2
        o = Oracle2D(H, Nh, ucuts(Nh, 2), Nh // 4, UNIT, dt)
        o.init()
        for _ in range(int(round(T / dt))):
            o.coarse_step()
            o.local_step()
        errs.append({nm: _broken(o, nm, T) for nm in ("pF", "pf", "pm", "u1", "u2")})
        perr.append(fe_errors(o.fg.mc, o.merged()["p"], exact("p", T), degree=1)[0])
    rate = lambda a, b: np.log(a / b) / np.log(4.0)
    for nm in ("pF", "pf", "pm", "u1", "u2"):
        assert rate(errs[0][nm][1], errs[1][nm][1]) > 0.9, (nm, errs)
    for nm in ("pf", "pm"):
        assert rate(errs[0][nm][0], errs[1][nm][0]) > 1.8, (nm, errs)
    assert rate(perr[0], perr[1]) > 0.9, perr


# --------------------------------------------------------------------------
# Porous part of Step 1 with non-unit parameters: convergence to Example 1
# --------------------------------------------------------------------------
def test_porous_step_converges_with_skewed_parameters():
    """Eqs. (5.1)-(5.3) (= Algorithm 1 Step 1) with every parameter different
    (phi_i C_i, k_i, mu_tilde, sigma, sigma*): the sources of Example 1 are
    derived for these parameters and the Gamma flux is set to the value the
    interface mass condition of Section 2 gives, u.n_c = (k_F / mu) dp_F/dy.
    The three pressures then converge to the exact ones at the P2 rates
    (L2 ~ h^3, H1 ~ h^2).  A dropped, swapped or mis-signed exchange term
    (s* between F and f, s between f and m) converges to a different solution
    and fails."""
    dypF = sp.lambdify((x, y, t), sp.diff(_EX["pF"], y), "numpy")
    dt, ns = 2e-4, 100
    T = dt * ns
    errs = []
    for N in (4, 8, 16):
        co = Coefs(SKEW, dt)
        mms = MMS(SKEW)
        gp = GridProblem(N, co)
        P = [interp_p2(gp.mp, mms, nm, 0.0) for nm in ("pF", "pf", "pm")]
        xc = gp.mc.p2_coords()
        n2 = gp.mc.n2 ** 2
        for n in range(ns):
            U = np.zeros(2 * n2)         # only the Gamma row of u_y is read
            U[n2:] = -(SKEW["k"][0] / SKEW["mu_tilde"]) * dypF(xc[:, 0], np.ones(n2), n * dt)
            P = porous_step(gp, mms, P, U, (n + 1) * dt)
        errs.append([fe_errors(gp.mp, P[i], exact(nm, T)) for i, nm in enumerate(("pF", "pf", "pm"))])
    e = np.array(errs)                  # (level, field, norm)
    rates = np.log2(e[:-1] / e[1:])
    # finest pair: the asymptotic rates; coarsest pair (N = 4 -> 8): p_m, the
    # steepest field, is still pre-asymptotic there
    assert (rates[-1, :, 0] > 2.7).all() and (rates[-1, :, 1] > 1.8).all(), rates
    assert (rates[:, :, 0] > 2.5).all() and (rates[:, :, 1] > 1.5).all(), rates


# --------------------------------------------------------------------------
# Exchange balance of the lagged porous equations
# --------------------------------------------------------------------------
def _exchange_balance(M, K, free, co, Pold, Pnew, Q):
    """Sum over the three porous equations, tested with the indicator of the
    free nodes, of everything except the exchange terms (Q holds the sources
    and, for p_F, the Gamma flux); returns it with the lag imbalance of the
    exchange terms and the size of the exchange flux.  The continuous exchange
    terms cancel in the sum (s*(pF - pf) + s*(pf - pF) + s(pf - pm) +
    s(pm - pf) = 0); the scheme lags p_f in the F equation, p_F and p_m in the
    f equation and p_f in the m equation, so the sum of its exchange terms is
    s* 1'M(dP_F + dP_f) + s 1'M(dP_f + dP_m), d = new - old."""
    one = free.astype(float)
    d = [Pnew[i] - Pold[i] for i in range(3)]
    rest = sum(one @ (co.tau[i] * (M @ d[i]) + co.kap[i] * (K @ Pnew[i]) - Q[i]) for i in range(3))
    lag = one @ (M @ (co.sst * (d[0] + d[1]) + co.s * (d[1] + d[2])))
    flux = one @ (M @ (co.sst * np.abs(Pnew[0] - Pnew[1]) + co.s * np.abs(Pnew[1] - Pnew[2])))
    return rest, lag, flux


def _porous_sources(grid, mms, t1, Uy):
    """Sources of the three porous equations at t1 on a grid, with the Gamma
    flux of u_y (conduit lattice) added to the p_F one."""
    E = np.arange(2 * grid.mp.N ** 2)
    Q = [forms.load_p2(grid.mp, E, lambda X, nm=nm: mms(nm, X, t1)) for nm in ("qF", "qf", "qm")]
    Q[0] = Q[0] - grid.Gp @ (grid.T_cp @ Uy)
    return Q


def test_exchange_balance_coarse_and_local():
    """Mass exchange between the three porosities is conservative in the model
    (Section 2: the exchange terms of the three equations cancel).  For the
    coarse porous step (Eqs. (5.1)-(5.3)) and for the local porous solves of
    Step 3 (1) (one subdomain per region, so the merged fine field is the
    local solution on all of Omega_p), the tested sum of the three equations
    without their exchange terms equals minus the lag imbalance
    s* 1'M(dP_F + dP_f) + s 1'M(dP_f + dP_m) to rounding.  The imbalance is
    small against the exchange flux and shrinks with dt."""
    NH, Nh = 2, 8
    cuts = {(r, a): [0, Nh] for r in (POROUS, CONDUIT) for a in (0, 1)}
    worst = {}
    for dt in (4e-2, 1e-2):
        o = Oracle2D(NH, Nh, cuts, 0, SKEW, dt)
        o.init()
        ratios = []
        for step in range(3):
            Pc_old, Uc_old = [p.copy() for p in o.P], o.U.copy()
            fine_old = o.merged() if step > 0 else None
            o.coarse_step()
            o.local_step()
            t1 = o.t(o.n)
            cg, fg = o.cg, o.fg
            Q = _porous_sources(cg, o.mms, t1, Uc_old[cg.mc.n2 ** 2:])
            rest, lag, flux = _exchange_balance(cg.M, cg.K, ~cg.dir_p, o.co, Pc_old, o.P, Q)
            assert abs(rest + lag) < 1e-12 * max(1.0, abs(rest), flux), (rest, lag)
            ratios.append(abs(lag) / flux)
            if fine_old is None:
                continue
            m = o.merged()
            Q = _porous_sources(fg, o.mms, t1, o._pro["U0"][fg.mc.n2 ** 2:])
            Pold = [fine_old[k] for k in ("pF", "pf", "pm")]
            Pnew = [m[k] for k in ("pF", "pf", "pm")]
            rest, lag, flux = _exchange_balance(fg.M, fg.K, ~fg.dir_p, o.co, Pold, Pnew, Q)
            assert abs(rest + lag) < 1e-12 * max(1.0, abs(rest), flux), (rest, lag)
            ratios.append(abs(lag) / flux)
        worst[dt] = max(ratios)
    assert worst[4e-2] < 0.5 and worst[1e-2] < 0.5 * worst[4e-2], worst


# --------------------------------------------------------------------------
# Overlap (Algorithm 3 Step 2) and linearity
# --------------------------------------------------------------------------
def test_overlap_monotonicity():
    """Step 2 enlarges each core D_j by the overlap.  Against the
    single-subdomain run (one Omega = the whole region: the local problem is
    then the fine problem itself), the porous fields' difference falls
    strictly as the overlap grows (the artificial boundary, where the local
    correction is pinned to zero, moves away from the core).  The conduit
    fields are not monotone in the overlap: their local pressure level comes
    from the coarse pressure on the artificial faces, whose accuracy depends
    on where the faces cut the coarse cells; they still end far below where
    they start."""
    prm = dict(UNIT, nu=0.1, k=[0.5, 0.2, 0.05], sigma=2.0)
    NH, Nh, dt, ns = 4, 16, 0.01, 3

    def run(cuts, ov):
        o = Oracle2D(NH, Nh, cuts, ov, prm, dt)
        o.init()
        for _ in range(ns):
            o.coarse_step()
            o.local_step()
        return o.merged()
    ref = run({(r, a): [0, Nh] for r in (POROUS, CONDUIT) for a in (0, 1)}, 0)
    mp, mc = RegionMesh(Nh, POROUS), RegionMesh(Nh, CONDUIT)
    d = []
    for ov in (1, 2, 4, 8):
        m = run(ucuts(Nh, 4), ov)
        d.append([rel_mass(mp, m[k], ref[k]) for k in ("pF", "pf", "pm")] + [rel_mass(mc, m["u"], ref["u"], ncomp=2)])
    d = np.array(d)
    assert (d[1:, :3] < d[:-1, :3]).all(), d
    assert d[-1, 3] < 0.5 * d[0, 3], d


def test_linearity_without_convection():
    """With the convection term off (Stokes conduit), every step of Algorithm 3
    is linear in the data (forcing, boundary and initial values): data
    a + 2 b gives solution(a) + 2 solution(b), coarse and merged."""
    NH, Nh, dt = 2, 8, 0.05
    prm = dict(SKEW, nu=0.2)
    ma, mb = MMS(prm), MMS(dict(prm, nu=0.7, sigma=1.5))
    data = {"a": lambda nm, X, tt: ma(nm, X, tt),
            "b": lambda nm, X, tt: mb(nm, X, tt + 0.7) * 0.5,
            "ab": lambda nm, X, tt: ma(nm, X, tt) + mb(nm, X, tt + 0.7)}
    res = {}
    for key, fn in data.items():
        o = Oracle2D(NH, Nh, ucuts(Nh, 2), 1, prm, dt, convection=False)
        o.mms = fn
        o.init()
        for _ in range(2):
            o.coarse_step()
            o.local_step()
        res[key] = (o.merged(), o.coarse())
    for lvl in (0, 1):
        for k in res["a"][lvl]:
            a, b, ab = res["a"][lvl][k], res["b"][lvl][k], res["ab"][lvl][k]
            assert np.abs(ab - (a + 2 * b)).max() < 1e-11 * np.abs(ab).max(), (lvl, k)
