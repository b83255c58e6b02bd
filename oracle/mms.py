"""Manufactured solution of Example 1 (Section 6, 2D experimental rate of
convergence) and the data the scheme needs from it: source terms q_F, q_f, q_m
and f_c of the model equations (Section 2, Eqs. for p_F, p_f, p_m and the
transient Navier-Stokes system), Dirichlet data and initial values.

The source terms are derived symbolically (sympy) from the model's strong form
with the run's parameters, so that the exact solution satisfies the PDEs in
the interior for any parameter set.  With non-unit parameters the interface
conditions are generally not satisfied by this solution; the scheme is run as
written and only takes sources, boundary and initial data from it.
"""
import numpy as np
import sympy as sp

x, y, t = sp.symbols("x y t", real=True)


def exact_ex1():
    """Example 1 exact fields as sympy expressions (p_m, p_f, p_F, u_c, p)."""
    g = 2 - sp.pi * sp.sin(sp.pi * x)
    pm = g * sp.sin(sp.Rational(1, 2) * sp.pi * (3 * y**3 - 2 * y**2)) * sp.cos(t)
    pf = g * sp.cos(sp.pi * (1 - y)) * sp.cos(t)
    pF = g * (1 - y - sp.cos(sp.pi * y)) * sp.cos(t)
    u1 = (x**2 * (y - 1)**2 + y) * sp.cos(t)
    u2 = -sp.Rational(2, 3) * x * (y - 1)**3 * sp.cos(t) + g * sp.cos(t)
    p = g * sp.sin(sp.Rational(1, 2) * sp.pi * y) * sp.cos(t)
    return dict(pF=pF, pf=pf, pm=pm, u1=u1, u2=u2, p=p)


def sources(ex, prm):
    """Strong-form sources for the given parameters (dict of floats).

    q_F = phi_F C_F dpF/dt - div(k_F/mu grad pF) + s*(pF - pf)
    q_f = phi_f C_f dpf/dt - div(k_f/mu grad pf) + s*(pf - pF) + s(pf - pm)
    q_m = phi_m C_m dpm/dt - div(k_m/mu grad pm) + s(pm - pf)
    f   = du/dt - div(2 nu D(u) - p I) + (u . grad) u
    with s* = sigma* k_f / mu and s = sigma k_m / mu.
    """
    mu = prm["mu_tilde"]
    kF, kf, km = prm["k"]
    sst = prm["sigma_star"] * kf / mu
    s = prm["sigma"] * km / mu
    phC = [prm["phi"][i] * prm["C"][i] for i in range(3)]
    lap = lambda e: sp.diff(e, x, 2) + sp.diff(e, y, 2)
    pF, pf, pm = ex["pF"], ex["pf"], ex["pm"]
    qF = phC[0] * sp.diff(pF, t) - kF / mu * lap(pF) + sst * (pF - pf)
    qf = phC[1] * sp.diff(pf, t) - kf / mu * lap(pf) + sst * (pf - pF) + s * (pf - pm)
    qm = phC[2] * sp.diff(pm, t) - km / mu * lap(pm) + s * (pm - pf)
    u = [ex["u1"], ex["u2"]]
    X = [x, y]
    nu = prm["nu"]
    f = []
    for c in range(2):
        # -div(2 nu D(u))_c = -nu sum_j d_j (d_j u_c + d_c u_j)
        visc = -nu * sum(sp.diff(sp.diff(u[c], X[j]) + sp.diff(u[j], X[c]), X[j]) for j in range(2))
        conv = sum(u[j] * sp.diff(u[c], X[j]) for j in range(2))
        f.append(sp.diff(u[c], t) + visc + sp.diff(ex["p"], X[c]) + conv)
    return dict(qF=qF, qf=qf, qm=qm, f1=f[0], f2=f[1])


class MMS:
    """Numerical callables f(xy (n,2), t) -> (n,) for exact fields and sources."""

    def __init__(self, prm):
        ex = exact_ex1()
        src = sources(ex, prm)
        self.expr = dict(ex, **src)
        self.fn = {k: sp.lambdify((x, y, t), v, "numpy") for k, v in self.expr.items()}

    def __call__(self, name, xy, tt):
        v = self.fn[name](xy[:, 0], xy[:, 1], tt)
        return np.broadcast_to(np.asarray(v, dtype=np.float64), (xy.shape[0],)).copy()
