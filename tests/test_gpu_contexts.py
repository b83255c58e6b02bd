"""Two live contexts with different parameters in one process: each keeps its
own coefficients, so stepping them in turn gives, bit for bit, what each
gives alone, and each still matches the oracle."""
import numpy as np
import pytest

from paper_2311_05170_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("pF", "pf", "pm", "u", "p")


def _make(cfg, precision):
    from paper_2311_05170_amd.lib import LocalParallel
    return LocalParallel(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], cfg["prm"], cfg["dt"],
                         cuts=W.flat_cuts(cfg["cuts"]), precision=precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_interleaved_contexts_keep_their_parameters(precision):
    a_cfg = W.small(dt=0.05)
    b_cfg = W.small(dt=0.02, prm=dict(W.unit_params(), nu=0.05, k=[0.3, 0.02, 0.005], sigma=4.0,
                                      sigma_star=0.2, alpha=0.7))
    steps = 3
    solo = {}
    for name, cfg in (("a", a_cfg), ("b", b_cfg)):
        g = _make(cfg, precision)
        for _ in range(steps):
            g.step()
        solo[name] = {f: g.solution(f) for f in FIELDS}
        g.close()
    ga, gb = _make(a_cfg, precision), _make(b_cfg, precision)
    try:
        for _ in range(steps):
            ga.step()
            gb.step()
        for name, g in (("a", ga), ("b", gb)):
            for f in FIELDS:
                assert np.array_equal(g.solution(f), solo[name][f]), (name, f)
    finally:
        ga.close()
        gb.close()
    # and each against the oracle after the same steps
    from oracle.scheme import Oracle2D
    for name, cfg in (("a", a_cfg), ("b", b_cfg)):
        o = Oracle2D(cfg["NH"], cfg["Nh"], cfg["cuts"], cfg["overlap"], cfg["prm"], cfg["dt"])
        o.init()
        for _ in range(steps):
            o.coarse_step()
            o.local_step()
        ref = o.merged()
        for f in FIELDS:
            err = np.abs(solo[name][f] - ref[f]).max() / np.abs(ref[f]).max()
            assert err < (1e-9 if precision == "fp64" else 1e-7), (name, f, err)
