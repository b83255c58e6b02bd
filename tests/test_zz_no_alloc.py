"""lp_local_step_noalloc (the local step with its refinement scratch in a
static device array instead of context buffers) against lp_local_step: two
contexts with the same inputs, one stepped by each entry point, give the same
fields; then again with a smaller problem, so the second use of the static
array starts from the first one's leftovers."""
import ctypes

import numpy as np
import pytest

from paper_2311_05170_amd import workloads as W

pytestmark = pytest.mark.gpu


def _make(cfg, precision, samples=None):
    from paper_2311_05170_amd.lib import LocalParallel
    return LocalParallel(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], cfg["prm"], cfg["dt"],
                         cuts=W.flat_cuts(cfg["cuts"]), precision=precision, samples=samples)


def _fields(g, nsub, nsamples=1):
    out = {}
    for smp in range(nsamples):
        for f in ("u", "p", "pF", "pf", "pm"):
            out[(smp, f)] = g.solution(f, sample=smp)
        for sub in range(nsub):
            for f in (("pF", "pf", "pm") if sub < nsub // 2 else ("u", "p")):
                out[(smp, sub, f)] = g.solution(f, "local", sub, sample=smp)
    return out


def _run_pair(cfg, precision, steps, samples=None):
    from paper_2311_05170_amd import lib
    fn = lib._LIB.lp_local_step_noalloc
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    fn.restype = ctypes.c_int32
    a, b = _make(cfg, precision, samples), _make(cfg, precision, samples)
    for _ in range(steps):
        a.coarse_step()
        a.local_step()
        b.coarse_step()
        lib._check(fn(b._h, b._s()))
    nsub = 2 * cfg["nsub"][0] * cfg["nsub"][1]
    S = len(samples) if samples else 1
    fa, fb = _fields(a, nsub, S), _fields(b, nsub, S)
    sa, sb = a.stats(), b.stats()
    a.close()
    b.close()
    for k in fa:
        scale = max(float(np.max(np.abs(fa[k]))), 1e-300)
        assert np.max(np.abs(fa[k] - fb[k])) <= 1e-12 * scale, k
    assert sa["flags"] == 0 and sb["flags"] == 0, (sa, sb)
    assert sa["ir_sweeps_max"] == sb["ir_sweeps_max"], (sa, sb)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_local_step_matches_local_step(precision):
    big = W.small(NH=3, refine=4, nsub=3, overlap=1, dt=0.02,
                  prm=dict(W.unit_params(), nu=0.05, k=[0.3, 0.02, 0.004], sigma=2.0, sigma_star=0.5))
    _run_pair(big, precision, 3)
    _run_pair(W.small(), precision, 2)         # smaller second use of the same array


def test_noalloc_local_step_with_samples():
    """Several samples in one context: the static array holds every sample's
    refinement scratch; same fields as lp_local_step, then a smaller
    single-sample problem on the same array."""
    cfg = dict(W.small(NH=3, refine=4, nsub=3, overlap=1), dt=0.01)
    _run_pair(cfg, "mixed", 3, samples=W.ensemble_samples(3))
    _run_pair(W.small(), "mixed", 2)
