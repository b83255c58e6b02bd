"""Manufactured solution of Example 2 (Section 6, 3D experimental rate of
convergence), reflected onto the unit-cube regions used here, and the data the
scheme needs from it.

The paper places the conduit below the interface (z <= 0) and the triple-
porosity region above it (z >= 0).  Here the porous region is (0,1)^3 below
the conduit (0,1)^2 x (1,2), so the paper's fields are evaluated at
z_p = 1 - z: pressures p_i(x, y, z) = p_i^paper(x, y, 1 - z) and
u = (u_1, u_2, -u_3)^paper(x, y, 1 - z).  The reflection maps the model onto
itself (the vertical velocity and every normal change sign together), so the
reflected fields satisfy the same equations and interface conditions.

Sources are derived symbolically from the strong form with the run's
parameters, as for Example 1.
"""
import numpy as np
import sympy as sp

x, y, z, t = sp.symbols("x y z t", real=True)


def exact_ex2_paper(zp):
    """Example 2's fields in the paper's coordinates, as expressions of x, y,
    zp (the paper's vertical coordinate) and t."""
    e = sp.exp(-t)
    s, c = sp.sin(x * y), sp.cos(x * y)
    r2 = x**2 + y**2
    pm = -zp + sp.exp(zp) - e * s * sp.cos(zp)
    pf = -zp + sp.exp(zp) - e * s * sp.cos(zp)
    pF = -zp + (-r2 + 8) * e * s * sp.cos(zp)
    u1 = (2 * x * s + y * (r2 - 8) * c) * e
    u2 = (2 * y * s + x * (r2 - 8) * c) * e
    u3 = 1 + (r2 * (r2 - 8) * s - 4 * s - 8 * x * y * c) * zp * e
    p = (-16 * x * y * c + (r2 + zp**2 - 8) * (2 * r2 + 2 * zp**2 - 1) * s - 8 * s) * e
    return dict(pF=pF, pf=pf, pm=pm, u1=u1, u2=u2, u3=u3, p=p)


def exact_ex2():
    """The reflected fields (z = 1 - z_p, u_3 sign flipped) in this build's
    coordinates."""
    zp = sp.Symbol("zp", real=True)
    ex = exact_ex2_paper(zp)
    out = {k: v.subs(zp, 1 - z) for k, v in ex.items()}
    out["u3"] = -out["u3"]
    return out


def sources3(ex, prm):
    """Strong-form sources for the given parameters (dict of floats), as
    Example 1's in 3D:
    q_i = phi_i C_i dp_i/dt - div(k_i/mu grad p_i) + exchange terms,
    f = du/dt - div(2 nu D(u) - p I) + (u . grad) u."""
    mu = prm["mu_tilde"]
    kF, kf, km = prm["k"]
    sst = prm["sigma_star"] * kf / mu
    s = prm["sigma"] * km / mu
    phC = [prm["phi"][i] * prm["C"][i] for i in range(3)]
    X = [x, y, z]
    lap = lambda e: sum(sp.diff(e, v, 2) for v in X)  # noqa: E731
    pF, pf, pm = ex["pF"], ex["pf"], ex["pm"]
    qF = phC[0] * sp.diff(pF, t) - kF / mu * lap(pF) + sst * (pF - pf)
    qf = phC[1] * sp.diff(pf, t) - kf / mu * lap(pf) + sst * (pf - pF) + s * (pf - pm)
    qm = phC[2] * sp.diff(pm, t) - km / mu * lap(pm) + s * (pm - pf)
    u = [ex["u1"], ex["u2"], ex["u3"]]
    nu = prm["nu"]
    f = []
    for c in range(3):
        visc = -nu * sum(sp.diff(sp.diff(u[c], X[j]) + sp.diff(u[j], X[c]), X[j]) for j in range(3))
        conv = sum(u[j] * sp.diff(u[c], X[j]) for j in range(3))
        f.append(sp.diff(u[c], t) + visc + sp.diff(ex["p"], X[c]) + conv)
    return dict(qF=qF, qf=qf, qm=qm, f1=f[0], f2=f[1], f3=f[2])


def example2_params():
    """Example 2's parameters: every parameter 1 except k_m = 0.01."""
    return dict(phi=[1.0] * 3, C=[1.0] * 3, k=[1.0, 1.0, 0.01], mu_tilde=1.0, sigma=1.0, sigma_star=1.0,
                rho=1.0, alpha=1.0, eta=1.0, nu=1.0)


class MMS3:
    """Numerical callables f(xyz (n,3), t) -> (n,) for exact fields and sources."""

    def __init__(self, prm):
        ex = exact_ex2()
        src = sources3(ex, prm)
        self.expr = dict(ex, **src)
        self.fn = {k: sp.lambdify((x, y, z, t), v, "numpy") for k, v in self.expr.items()}

    def __call__(self, name, xyz, tt):
        v = self.fn[name](xyz[:, 0], xyz[:, 1], xyz[:, 2], tt)
        return np.broadcast_to(np.asarray(v, dtype=np.float64), (xyz.shape[0],)).copy()
