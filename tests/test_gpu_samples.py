"""Parameter samples advanced together (lp_options.nsamples > 1): every launch
covers the systems of all samples, and each sample's fields are, bit for bit,
what a context holding that sample alone computes (the same kernels, reduction
orders and Newton/refinement decisions per sample), which the one-sample
tests pin to the oracle.  The small case is also checked against the oracle
directly, sample by sample."""
import numpy as np
import pytest

from paper_2311_05170_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("pF", "pf", "pm", "u", "p")


def _make(cfg, samples, precision, **kw):
    from paper_2311_05170_amd.lib import LocalParallel
    return LocalParallel(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], samples[0], cfg["dt"],
                         cuts=W.flat_cuts(cfg["cuts"]), precision=precision, samples=samples, **kw)


def _fields(g, sample, subs):
    out = {}
    for f in FIELDS:
        out[f, "merged"] = g.solution(f, sample=sample)
        out[f, "coarse"] = g.solution(f, "coarse", sample=sample)
    for sub in subs:
        for f in (("pF", "pf", "pm") if sub < g.n_sub // 2 else ("u", "p")):
            out[f, "local", sub] = g.solution(f, "local", sub, sample=sample)
    return out


def _compare(cfg, samples, precision, steps, check):
    """Step an ensemble context and one context per checked sample; compare
    every field bit for bit after each step."""
    ens = _make(cfg, samples, precision)
    solo = {i: _make(cfg, [samples[i]], precision) for i in check}
    try:
        n_sub = ens.n_sub
        subs = (0, n_sub // 2 - 1, n_sub // 2, n_sub - 1)
        for k in range(steps):
            ens.step()
            for g in solo.values():
                g.step()
            for i, g in solo.items():
                a, b = _fields(ens, i, subs), _fields(g, 0, subs)
                for key in b:
                    assert np.isfinite(b[key]).all(), (precision, k, i, key)
                    assert np.array_equal(a[key], b[key]), (precision, k, i, key,
                                                            np.abs(a[key] - b[key]).max())
        st = ens.stats()
        one = next(iter(solo.values())).stats()
        # per-sample statistics: those of the sample's own context
        for i, g in solo.items():
            a, b = ens.stats(sample=i), g.stats()
            for key in ("newton_its", "newton_its_max", "ir_sweeps", "ir_relres", "ir_sweeps_porous",
                        "ir_relres_porous", "ir_sweeps_oseen", "ir_relres_oseen", "local_dofs"):
                assert a[key] == b[key], (i, key, a[key], b[key])
            assert (a["flags"] & 2) == (b["flags"] & 2), (i, a["flags"], b["flags"])
        assert st["flags"] == 0, st
        assert st["n_porous"] == one["n_porous"] and st["n_conduit"] == one["n_conduit"]
        assert st["local_dofs"] == len(samples) * one["local_dofs"]
        assert st["newton_its_max"] >= max(g.stats()["newton_its_max"] for g in solo.values())
        g0 = next(iter(solo.values()))
        for which, sub in ((0, 0), (1, 0), (3, n_sub - 1), (4, n_sub - 1), (5, 0)):
            assert np.array_equal(ens.index_map(which, sub), g0.index_map(which, sub)), which
        with pytest.raises(Exception, match="sample out of range"):
            ens.solution("u", sample=len(samples))
        with pytest.raises(Exception, match="sample out of range"):
            ens.stats(sample=len(samples))
    finally:
        ens.close()
        for g in solo.values():
            g.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_samples_match_single_sample_contexts_small(precision):
    cfg = W.small(dt=0.05)
    samples = W.ensemble_samples(3)
    _compare(cfg, samples, precision, 3, check=(0, 1, 2))


@pytest.mark.parametrize("precision", ["mixed"])
def test_samples_match_single_sample_contexts_cfg1(precision):
    cfg = dict(W.config("cfg1"), dt=0.01)          # the ensemble's time step
    samples = W.ensemble_samples(5, seed=11)
    _compare(cfg, samples, precision, 2, check=(0, 4))


def test_ensemble_workload_sampled():
    """The benchmarked ensemble (cfg2 geometry, 32 samples, mixed precision):
    the first, the last and the one of smallest viscosity against their own
    contexts."""
    cfg = W.ensemble()
    _compare(cfg, cfg["samples"], "mixed", 2, check=(0, 18, 31))   # 18: the smallest nu


def test_samples_match_oracle_small():
    from oracle.scheme import Oracle2D
    cfg = W.small(dt=0.05)
    samples = W.ensemble_samples(3)
    steps = 3
    g = _make(cfg, samples, "fp64")
    try:
        for _ in range(steps):
            g.step()
        got = {i: {f: g.solution(f, sample=i) for f in FIELDS} for i in range(len(samples))}
    finally:
        g.close()
    for i, prm in enumerate(samples):
        o = Oracle2D(cfg["NH"], cfg["Nh"], cfg["cuts"], cfg["overlap"], prm, cfg["dt"])
        o.init()
        for _ in range(steps):
            o.coarse_step()
            o.local_step()
        ref = o.merged()
        for f in FIELDS:
            err = np.abs(got[i][f] - ref[f]).max() / np.abs(ref[f]).max()
            print("sample", i, f, "%.1e" % err, flush=True)
            assert err < 1e-9, (i, f, err)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_samples_under_hip_graphs(precision):
    """Several samples with every step's launch sequences replayed as HIP
    graphs: the same fields, bit for bit, as direct launches (graphs start at
    the third step; eight steps replay every ring slot's graphs at least once)."""
    cfg = dict(W.config("cfg1"), dt=0.01)
    samples = W.ensemble_samples(4, seed=3)
    a, b = _make(cfg, samples, precision), _make(cfg, samples, precision, graphs=True)
    try:
        for k in range(10):
            a.step()
            b.step()
            for i in range(len(samples)):
                for f in FIELDS:
                    x, y = a.solution(f, sample=i), b.solution(f, sample=i)
                    assert np.array_equal(x, y), (precision, k, i, f, np.abs(x - y).max())
        assert a.stats()["flags"] == 0 and b.stats()["flags"] == 0
    finally:
        a.close()
        b.close()


def test_samples_with_autotuning():
    """The autotuner on a context of several samples tunes the dense path (the
    factorisation variant and solve depth over all samples' systems); the
    fields stay at oracle parity, as the small case's fixed variants are."""
    from oracle.scheme import Oracle2D
    cfg = W.small(dt=0.05)
    samples = W.ensemble_samples(3)
    steps = 3
    g = _make(cfg, samples, "mixed", autotune=True)
    try:
        for _ in range(steps):
            g.step()
        st = g.stats()
        assert st["tuned"] == 1 and st["solver"] == 1 and st["flags"] == 0, st
        got = {i: {f: g.solution(f, sample=i) for f in FIELDS} for i in range(len(samples))}
    finally:
        g.close()
    for i, prm in enumerate(samples):
        o = Oracle2D(cfg["NH"], cfg["Nh"], cfg["cuts"], cfg["overlap"], prm, cfg["dt"])
        o.init()
        for _ in range(steps):
            o.coarse_step()
            o.local_step()
        ref = o.merged()
        for f in FIELDS:
            err = np.abs(got[i][f] - ref[f]).max() / np.abs(ref[f]).max()
            assert err < 1e-7, (i, f, err)
