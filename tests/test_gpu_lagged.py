"""LP_LAG_MERGED (the lagged e^n of Eqs. (5.5)-(5.8) taken from the merged
correction of Step 4) against the oracle's Algorithm 3 with the same reading:
merged fields, coarse fields and every subdomain's correction after every
step, to the same bounds as the default reading's parity tests; and the
default reading left as it was."""
import numpy as np
import pytest

from oracle.scheme import Oracle2D
from paper_2311_05170_amd import workloads as W
from test_gpu_parity import TOL, ELEM_TOL, _gpu, compare, elementwise, local_corrections

pytestmark = pytest.mark.gpu


def _run(cfg, precision, steps, samples=None):
    o = Oracle2D(cfg["NH"], cfg["Nh"], cfg["cuts"], cfg["overlap"], cfg["prm"], cfg["dt"], previous="merged")
    o.init()
    g = _gpu(cfg, precision, lagged="merged")
    try:
        for n in range(steps):
            o.coarse_step()
            g.coarse_step()
            ec = compare(o, g, "coarse")
            o.local_step()
            g.local_step()
            em = compare(o, g, "merged")
            ee = elementwise(o, g)
            el = local_corrections(o, g)
            print("lagged merged", precision, "step", n + 1, {k: "%.1e" % v for k, v in em.items()},
                  {k: "%.1e" % v for k, v in ee.items()}, {k: "%.1e" % v for k, v in el.items()}, flush=True)
            assert max(ec.values()) < 1e-10, ec
            assert max(em.values()) < TOL[precision], em
            assert max(ee.values()) < ELEM_TOL[precision], ee
            assert max(el.values()) < ELEM_TOL[precision], el
        assert g.stats()["flags"] == 0
    finally:
        g.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lagged_merged_small(precision):
    """2 x 2 subdomains per region, H = 1/2, h = 1/8, unit parameters."""
    _run(W.small(), precision, 3)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lagged_merged_shifted_cuts(precision):
    """Uneven cores from shifted cut lines: corrections of neighbours with
    different boxes meet on every seam."""
    _run(W.shifted_small(), precision, 3)


def test_lagged_merged_cfg1():
    """cfg1 (H = 1/4, h = 1/16, 4 x 4 + 4 x 4 subdomains), mixed, 2 steps."""
    _run(dict(W.config("cfg1"), dt=0.05), "mixed", 2)


def test_lagged_merged_with_samples_matches_solo_contexts():
    """Three samples in one context with LP_LAG_MERGED take the same path as
    three single-sample contexts, bit for bit."""
    from paper_2311_05170_amd.lib import LocalParallel
    cfg = dict(W.small(), dt=0.01)
    samples = W.ensemble_samples(3)
    args = (cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"])
    g = LocalParallel(*args, samples[0], cfg["dt"], cuts=W.flat_cuts(cfg["cuts"]), precision="mixed",
                      samples=samples, lagged="merged")
    solo = [LocalParallel(*args, s, cfg["dt"], cuts=W.flat_cuts(cfg["cuts"]), precision="mixed", lagged="merged")
            for s in samples]
    try:
        for _ in range(3):
            g.step()
            for s in solo:
                s.step()
        for k, s in enumerate(solo):
            for f in ("pF", "pf", "pm", "u", "p"):
                assert np.array_equal(g.solution(f, sample=k), s.solution(f)), (k, f)
    finally:
        g.close()
        for s in solo:
            s.close()


def test_lagged_reading_changes_the_result_and_states_do_not_mix():
    """The two readings differ after the second step (the first uses e^0 in
    both), and a state saved under one is refused by a context of the other."""
    from paper_2311_05170_amd.lib import LpError
    cfg = W.small(dt=0.05)
    a, b = _gpu(cfg, "fp64"), _gpu(cfg, "fp64", lagged="merged")
    try:
        a.step()
        b.step()
        assert np.array_equal(a.solution("pF"), b.solution("pF"))
        a.step()
        b.step()
        assert not np.array_equal(a.solution("pF"), b.solution("pF"))
        with pytest.raises(LpError, match="lagged"):
            b.load_state(a.save_state())
    finally:
        a.close()
        b.close()
