"""Error measures: L2 and H1-seminorm distances between a finite element field
and an exact function (used for the convergence studies of Section 6), and
the mass-matrix norm used to compare two discrete fields."""
import numpy as np

from .fe import triangle_rule, p2_basis, p1_basis
from . import forms

_PTS, _WTS = triangle_rule(6)
_P2V, _P2G = p2_basis(_PTS)
_P1V, _P1G = p1_basis(_PTS)


def fe_errors(mesh, vec, exact, degree=2, elems=None):
    """(L2 error, H1-seminorm error) of the P2 (degree=2) or P1 field `vec`
    against `exact(X) -> (values (n,), gradients (n,2))` over elements `elems`."""
    if elems is None:
        elems = np.arange(2 * mesh.N ** 2)
    e2 = 0.0
    g2 = 0.0
    for t in (0, 1):
        Et = elems[mesh.el_orient[elems] == t]
        if len(Et) == 0:
            continue
        J = mesh.jacobian(t)
        det = abs(np.linalg.det(J))
        invJ = np.linalg.inv(J)
        ci = mesh.el_cell[Et]
        v0 = np.stack([ci[:, 0] * mesh.h, mesh.y0 + ci[:, 1] * mesh.h], 1)
        X = v0[:, None, :] + np.einsum("kl,ql->qk", J, _PTS)[None]
        if degree == 2:
            ve = vec[mesh.el_p2[Et]]
            uh = ve @ _P2V.T
            gh = np.einsum("ea,qak->eqk", ve, _P2G @ invJ)
        else:
            ve = vec[mesh.el_p1[Et]]
            uh = ve @ _P1V.T
            gh = np.einsum("ea,ak->ek", ve, _P1G @ invJ)[:, None, :].repeat(len(_WTS), 1)
        ux, gx = exact(X.reshape(-1, 2))
        ux = ux.reshape(uh.shape)
        gx = gx.reshape(gh.shape)
        w = _WTS * det
        e2 += np.sum(w[None] * (uh - ux) ** 2)
        g2 += np.sum(w[None, :, None] * (gh - gx) ** 2)
    return np.sqrt(e2), np.sqrt(g2)


def mass_norm(mesh, vec, degree=2):
    """sqrt(v^T M v) with the region's P2 (or P1) mass matrix."""
    E = np.arange(2 * mesh.N ** 2)
    if degree == 2:
        M, _ = forms.p2_mass_stiff(mesh, E)
    else:
        M = forms.p1_mass(mesh, E)
    return float(np.sqrt(max(vec @ (M @ vec), 0.0)))
