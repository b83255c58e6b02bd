"""Algorithm 1 (Section 3.3, partitioned time stepping on one grid) on the
GPU (lp_options.scheme = LP_ONE_GRID) against the oracle's Algorithm 1 on the
same grid: every field after every step, in the relative mass norm and
element by element (FP64: <= 1e-9)."""
import numpy as np
import pytest

from oracle.norms import mass_norm
from oracle.scheme import algorithm1
from paper_2311_05170_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _rel(mesh, a, b, degree=2, ncomp=1):
    n = len(a) // ncomp
    num = sum(mass_norm(mesh, a[i * n:(i + 1) * n] - b[i * n:(i + 1) * n], degree) ** 2 for i in range(ncomp))
    den = sum(mass_norm(mesh, b[i * n:(i + 1) * n], degree) ** 2 for i in range(ncomp))
    return np.sqrt(num / max(den, 1e-300))


def _cfg2_params():
    return W.config("cfg2")["prm"]


@pytest.mark.parametrize("N,prm_fn,dt,steps", [(8, W.unit_params, 0.05, 3), (16, W.unit_params, 0.1, 3),
                                               (12, _cfg2_params, 0.01, 3)])
def test_one_grid_matches_oracle_algorithm1(N, prm_fn, dt, steps):
    from paper_2311_05170_amd.lib import LocalParallel
    prm = prm_fn()
    g = LocalParallel(N, 1, (2, 2), 1, prm, dt, precision="fp64", scheme="one_grid")
    try:
        for k in range(1, steps + 1):
            g.step()
            gp, ref = algorithm1(N, prm, dt, k)
            worst = {}
            for f in ("pF", "pf", "pm"):
                a = g.solution(f)
                worst[f] = (_rel(gp.mp, a, ref[f]), np.abs(a - ref[f]).max() / np.abs(ref[f]).max())
            a = g.solution("u")
            worst["u"] = (_rel(gp.mc, a, ref["u"], ncomp=2), np.abs(a - ref["u"]).max() / np.abs(ref["u"]).max())
            a = g.solution("p")
            worst["p"] = (_rel(gp.mc, a, ref["p"], degree=1), np.abs(a - ref["p"]).max() / np.abs(ref["p"]).max())
            print("N", N, "step", k, {f: "%.1e/%.1e" % v for f, v in worst.items()}, flush=True)
            for f, (r, e) in worst.items():
                assert r <= TOL and e <= TOL, (N, k, f, r, e)
            # the merged level is the one grid's, the coarse level the same
            assert np.array_equal(g.solution("u"), g.solution("u", "coarse"))
        st = g.stats()
        assert st["flags"] == 0 and st["step"] == steps, st
    finally:
        g.close()


def test_one_grid_has_no_local_level():
    from paper_2311_05170_amd.lib import LocalParallel, LpError
    g = LocalParallel(4, 1, (2, 2), 1, W.unit_params(), 0.1, precision="fp64", scheme="one_grid")
    try:
        g.step()
        with pytest.raises(LpError, match="no local corrections"):
            g.solution("u", "local", 0)
    finally:
        g.close()
