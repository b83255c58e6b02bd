"""Checkpoint and resume between steps (lp_save_state / lp_load_state): a
context set up with the same arguments that loads a state saved after step k
continues exactly as the saving context does, bit for bit in every field
(merged, coarse and local corrections), with the step count and the run-long
statistics carried over; states from other setups are refused."""
import numpy as np
import pytest

from paper_2311_05170_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("pF", "pf", "pm", "u", "p")


def _make(cfg, precision, samples=None, **kw):
    from paper_2311_05170_amd.lib import LocalParallel
    return LocalParallel(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], cfg["prm"], cfg["dt"],
                         cuts=W.flat_cuts(cfg["cuts"]), precision=precision, samples=samples, **kw)


def _fields(g, nsamples, local=True):
    out = {}
    for smp in range(nsamples):
        for f in FIELDS:
            out[smp, f, "merged"] = g.solution(f, sample=smp)
            out[smp, f, "coarse"] = g.solution(f, "coarse", sample=smp)
        if local:
            for sub in (0, g.n_sub // 2 - 1, g.n_sub // 2, g.n_sub - 1):
                for f in (("pF", "pf", "pm") if sub < g.n_sub // 2 else ("u", "p")):
                    out[smp, f, "local", sub] = g.solution(f, "local", sub, sample=smp)
    return out


CASES = [
    ("small", "fp64", None, {}, 3),
    ("cfg1", "mixed", None, {}, 3),
    # the Jacobian inverse in use is state: refreshed at steps 1, 4, 7, so
    # steps 5 and 6 after a save at step 4 run on the saved one
    ("cfg1", "mixed", None, {"jacobian_every": 3}, 4),
    ("small", "mixed", 3, {}, 3),                      # three samples in one context
    ("one_grid", "fp64", None, {}, 3),                 # Algorithm 1
]


@pytest.mark.parametrize("name,precision,nsamples,kw,first", CASES)
def test_resume_continues_bit_for_bit(name, precision, nsamples, kw, first):
    if name == "one_grid":
        cfg = dict(W.small(NH=8, refine=1, dt=0.05))
        kw = dict(kw, scheme="one_grid")
    else:
        cfg = W.small(dt=0.05) if name == "small" else dict(W.config("cfg1"), dt=0.05)
    samples = W.ensemble_samples(nsamples) if nsamples else None
    if samples:
        cfg = dict(cfg, dt=0.01)
    S = nsamples or 1
    more = 2
    a = _make(cfg, precision, samples, **kw)
    b = None
    try:
        for _ in range(first):
            a.step()
        state = a.save_state()
        before = _fields(a, S, local=name != "one_grid")
        for _ in range(more):
            a.step()
        want = _fields(a, S, local=name != "one_grid")
        want_st = a.stats()
        b = _make(cfg, precision, samples, **kw)
        b.load_state(state)
        # the loaded context reads back the saved step's fields at once
        got0 = _fields(b, S, local=name != "one_grid")
        for key in before:
            assert np.array_equal(got0[key], before[key]), key
        for _ in range(more):
            b.step()
        got = _fields(b, S, local=name != "one_grid")
        for key in want:
            assert np.array_equal(got[key], want[key]), (name, precision, key,
                                                         np.abs(got[key] - want[key]).max())
        st = b.stats()
        assert st["step"] == first + more == want_st["step"]
        for k in ("flags", "newton_its_max", "ir_sweeps_max", "ir_relres_max", "lu_growth_local",
                  "lu_pivot_local"):
            assert st[k] == want_st[k], (k, st[k], want_st[k])
    finally:
        a.close()
        if b is not None:
            b.close()


def test_foreign_or_damaged_states_are_refused():
    from paper_2311_05170_amd.lib import LpError
    cfg = W.small(dt=0.05)
    a = _make(cfg, "mixed")
    others = []
    try:
        a.step()
        state = a.save_state()
        a.coarse_step()
        with pytest.raises(LpError, match="pending"):
            a.save_state()
        with pytest.raises(LpError, match="pending"):
            a.load_state(state)
        a.local_step()
        # other parameters, other precision, other partition
        b = _make(dict(cfg, prm=dict(W.unit_params(), nu=0.5)), "mixed")
        others.append(b)
        with pytest.raises(LpError, match="other parameters"):
            b.load_state(state)
        c = _make(cfg, "fp64")
        others.append(c)
        with pytest.raises(LpError, match="another mesh"):
            c.load_state(state)
        d = _make(dict(W.small(dt=0.05, overlap=2)), "mixed")
        others.append(d)
        with pytest.raises(LpError):
            d.load_state(state)
        e = _make(cfg, "mixed")
        others.append(e)
        with pytest.raises(LpError, match="too short"):
            e.load_state(state[:len(state) // 2])
        with pytest.raises(LpError, match="not a saved state"):
            e.load_state(b"\0" * len(state))
        # a refused load leaves the context usable from its own start
        e.step()
        assert e.stats()["step"] == 1
    finally:
        a.close()
        for g in others:
            g.close()
