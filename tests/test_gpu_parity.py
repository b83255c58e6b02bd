"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle on the
same seeded inputs.  Merged fields are compared after every step in the
relative mass-matrix norm (<= 1e-8 for the FP64 path, <= 1e-7 for the mixed
path: FP32 factorisations won back by FP64 iterative refinement) and element
by element (max |gpu - oracle| / max |oracle| <= 1e-9 FP64, 1e-7 mixed); every
subdomain's correction e_j (Algorithm 3 Step 3, on its whole local lattice)
is compared element by element too."""
import functools
import os

import numpy as np
import pytest

from oracle.norms import mass_norm
from oracle.scheme import Oracle2D
from paper_2311_05170_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-8, "mixed": 1e-7}
# element-wise: max |gpu - oracle| over a field / max |oracle| over it
ELEM_TOL = {"fp64": 1e-9, "mixed": 1e-7}


def _gpu(cfg, precision, **kw):
    from paper_2311_05170_amd.lib import LocalParallel
    return LocalParallel(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], cfg["prm"], cfg["dt"],
                         cuts=W.flat_cuts(cfg["cuts"]), precision=precision, **kw)


def _oracle(cfg, **kw):
    o = Oracle2D(cfg["NH"], cfg["Nh"], cfg["cuts"], cfg["overlap"], cfg["prm"], cfg["dt"], **kw)
    o.init()
    return o


def rel(mesh, a, b, degree=2, ncomp=1):
    n = len(a) // ncomp
    num = sum(mass_norm(mesh, a[i * n:(i + 1) * n] - b[i * n:(i + 1) * n], degree) ** 2 for i in range(ncomp))
    den = sum(mass_norm(mesh, b[i * n:(i + 1) * n], degree) ** 2 for i in range(ncomp))
    return np.sqrt(num / max(den, 1e-300))


def compare(o, g, level):
    out = {}
    if level == "coarse":
        ref = o.coarse()
        mp, mc = o.cg.mp, o.cg.mc
    else:
        ref = o.merged()
        mp, mc = o.fg.mp, o.fg.mc
    for f in ("pF", "pf", "pm"):
        out[f] = rel(mp, g.solution(f, level), ref[f])
    out["u"] = rel(mc, g.solution("u", level), ref["u"], ncomp=2)
    out["p"] = rel(mc, g.solution("p", level), ref["p"], degree=1)
    return out


def elementwise(o, g):
    """max |gpu - oracle| / max |oracle| of every merged field."""
    ref = o.merged()
    return {f: float(np.max(np.abs(g.solution(f) - ref[f])) / max(np.max(np.abs(ref[f])), 1e-300))
            for f in ("pF", "pf", "pm", "u", "p")}


def local_corrections(o, g):
    """Worst element-wise difference of the subdomain corrections e_j (every
    subdomain, every node of its local lattice, Dirichlet nodes included),
    relative to the largest oracle value of that field over all subdomains."""
    from oracle.mesh import POROUS
    diff, scale = {}, {}
    for sd in o.subs:
        names = ("pF", "pf", "pm") if sd.region == POROUS else ("u", "p")
        ref = o.e[sd.sid]
        if sd.region == POROUS:
            pairs = [(names[i], g.solution(names[i], "local", sd.sid), ref[i]) for i in range(3)]
        else:
            pairs = [("u", g.solution("u", "local", sd.sid), np.concatenate([ref[0], ref[1]])),
                     ("p", g.solution("p", "local", sd.sid), ref[2])]
        for f, a, b in pairs:
            assert a.shape == b.shape, (sd.sid, f, a.shape, b.shape)
            diff[f] = max(diff.get(f, 0.0), float(np.max(np.abs(a - b))))
            scale[f] = max(scale.get(f, 0.0), float(np.max(np.abs(b))))
    return {f: diff[f] / max(scale[f], 1e-300) for f in diff}


def run_parity(cfg, precision, steps, locals_every_step=True, keep=False, **kw):
    o = _oracle(cfg, **{k: v for k, v in kw.items() if k == "convection"})
    g = _gpu(cfg, precision, **kw)
    worst = 0.0
    for n in range(steps):
        o.coarse_step()
        g.coarse_step()
        ec = compare(o, g, "coarse")
        o.local_step()
        g.local_step()
        em = compare(o, g, "merged")
        ee = elementwise(o, g)
        el = local_corrections(o, g) if (locals_every_step or n == steps - 1) else {}
        print("step", n + 1, "coarse", {k: "%.1e" % v for k, v in ec.items()},
              "merged", {k: "%.1e" % v for k, v in em.items()},
              "elementwise", {k: "%.1e" % v for k, v in ee.items()},
              "e_j", {k: "%.1e" % v for k, v in el.items()}, g.stats(), flush=True)
        worst = max(worst, max(ec.values()), max(em.values()))
        assert max(ec.values()) < 1e-10, ec
        assert max(em.values()) < TOL[precision], em
        assert max(ee.values()) < ELEM_TOL[precision], ee
        if el:
            assert max(el.values()) < ELEM_TOL[precision], el
    # no refinement or coarse step ended unconverged, no bad pivot (sticky flags)
    st = g.stats()
    assert st["flags"] == 0, st
    if keep:
        return g
    g.close()
    return worst


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_small_unit(precision):
    """2 x 2 subdomains per region, H = 1/2, h = 1/8, unit parameters."""
    run_parity(W.small(), precision, 3)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_small_ragged(precision):
    """3 x 3 subdomains on 12 cells with overlap 1 (uneven boxes and a
    ragged band), non-unit parameters."""
    prm = dict(W.unit_params(), nu=0.05, k=[0.3, 0.02, 0.004], sigma=2.0, sigma_star=0.5)
    cfg = W.small(NH=3, refine=4, nsub=3, overlap=1, dt=0.02, prm=prm)
    run_parity(cfg, precision, 3)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_shifted_cuts(precision):
    """Explicit cut lines passed through the ABI: every interior cut of the
    4 x 4 partition shifted by a SplitMix64 draw in {-1, 0, 1} fine cells
    (the uneven-core recipe of the h = 1/256 workload at a size the oracle
    finishes in seconds), so cores and local systems all differ in size."""
    cfg = W.shifted_small()
    assert len({tuple(v) for v in cfg["cuts"].values()}) > 1
    run_parity(cfg, precision, 3)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_single_subdomain_per_region(precision):
    """The degenerate partition: one subdomain per region, so no artificial
    boundary and one owner per merged node (each local problem is its whole
    region on the fine mesh, with the coarse solution as lagged data)."""
    run_parity(W.small(NH=2, refine=4, nsub=1, overlap=1), precision, 3)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_extreme_parameters(precision):
    """Small viscosity (nu = 1e-3: convection-dominated local Oseen systems,
    factored without pivoting), permeabilities down to 1e-4 and strong
    exchange (sigma = 10, sigma* = 0.1): the FP32 factorisations of the mixed
    path are less accurate and the refinement must still reach the tolerance."""
    prm = dict(W.unit_params(), nu=1e-3, k=[1e-4, 1e-3, 1e-2], sigma=10.0, sigma_star=0.1)
    run_parity(W.small(NH=2, refine=4, nsub=2, overlap=1, dt=0.01, prm=prm), precision, 3)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_cfg1(precision):
    """The 2D FP64 workload: H = 1/4, h = 1/16, 4 x 4 + 4 x 4 subdomains,
    overlap H/2, dt = 0.1, T = 0.5 (all 5 steps)."""
    cfg = W.config("cfg1")
    run_parity(cfg, precision, cfg["steps"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_cfg2_first_steps(precision):
    """The mixed-vs-FP64 workload (H = 1/8, h = 1/64, 8 x 8 + 8 x 8 subdomains,
    seeded parameters) for its first two steps (the oracle's share)."""
    cfg = W.config("cfg2")
    run_parity(cfg, precision, 2)


FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg2_oracle_steps.npz")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg2_bench_window_matches_stored_oracle(precision):
    """cfg2 in the configuration bench.py times (two refinement sweeps
    launched in the mixed path, the coarse Jacobian every third step, at most
    ten chord steps), 25 steps issued back to back, checked after steps 12 and
    25 against the oracle's fields stored by tests/golden/make_cfg2_fixture.py:
    the whole warmup and timed window stays within tolerance, and no flag is
    raised on the way."""
    from oracle.mesh import RegionMesh
    ref = np.load(FIXTURE)
    cfg = W.config("cfg2")
    mp, mc = RegionMesh(cfg["Nh"], 0), RegionMesh(cfg["Nh"], 1)
    g = _gpu(cfg, precision, max_ir=2, jacobian_every=3, max_newton=10)
    for n in range(1, 26):
        g.step()
        if n in (12, 25):
            for f in ("pF", "pf", "pm", "u", "p"):
                a, b = g.solution(f), ref["merged_%d_%s" % (n, f)]
                mesh = mp if f in ("pF", "pf", "pm") else mc
                em = rel(mesh, a, b, degree=1 if f == "p" else 2, ncomp=2 if f == "u" else 1)
                ee = np.max(np.abs(a - b)) / np.max(np.abs(b))
                print("step", n, f, "mass %.1e elementwise %.1e" % (em, ee), flush=True)
                assert em < TOL[precision] and ee < ELEM_TOL[precision], (n, f, em, ee)
    for f in ("pF", "pf", "pm", "u", "p"):
        a, b = g.solution(f, "coarse"), ref["coarse_25_" + f]
        assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(b)), f
    st = g.stats()
    g.close()
    assert st["flags"] == 0 and st["ir_sweeps_max"] <= 2, st
    assert st["ir_relres_max"] <= (1e-10 if precision == "mixed" else 1e-12), st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("width", ["6", "16"])
def test_parity_krylov_cfg1(precision, width, monkeypatch):
    """The Krylov path of the local Oseen solves (Eq. (5.8)): FGMRES in FP64
    with the matrix-free operator, preconditioned by restricted additive
    Schwarz over strips whose Stokes-part band matrices were factored at
    setup.  Strips of at most 6 cells cut every 6-8 cell box of cfg1 into 2-4
    overlapping strips; 16 leaves one strip per box (the whole box's Stokes
    part).  All five steps against the oracle."""
    monkeypatch.setenv("LP_KRYLOV_STRIP", width)
    cfg = W.config("cfg1")
    g = run_parity(cfg, precision, cfg["steps"], solver="krylov", max_ir=4, keep=True)
    st = g.stats()
    g.close()
    assert st["solver"] == 2 and 1 <= st["krylov_its"] <= 4 * 30, st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_krylov_shifted_cuts(precision, monkeypatch):
    """The Krylov path on uneven cores (explicit shifted cuts), strips of at
    most 6 cells."""
    monkeypatch.setenv("LP_KRYLOV_STRIP", "6")
    run_parity(W.shifted_small(), precision, 3, solver="krylov", max_ir=4)


FIXTURE3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg3_oracle_sampled.npz")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg3_uneven_batch_matches_stored_oracle(precision):
    """The uneven h = 1/256 workload (16 x 16 + 16 x 16 subdomains with
    SplitMix64-shifted cuts, local systems of 1.6k-5.9k porous and 4.4k-12.9k
    Oseen unknowns, half-bandwidths to 399): the local Oseen systems go to the
    Krylov path (too wide for the band window) and the porous ones to the band
    factorisation, all in one launch per stage.  Two steps against the
    oracle's record (tests/golden/make_cfg3_fixture.py): the full coarse
    fields, and every 29th entry of each merged field element by element (the
    record holds each field's largest magnitude), plus each field's sum of
    squares."""
    ref = np.load(FIXTURE3)
    stride = int(ref["stride"])
    cfg = W.config("cfg3")
    g = _gpu(cfg, precision, max_ir=3)
    assert g.stats()["solver"] == 2
    for n in (1, 2):
        g.step()
        for f in ("pF", "pf", "pm", "u", "p"):
            c = g.solution(f, "coarse")
            assert np.max(np.abs(c - ref["coarse_%d_%s" % (n, f)])) <= 1e-10 * np.max(np.abs(c)), (n, f)
            a = g.solution(f)
            ee = np.max(np.abs(a[::stride] - ref["merged_%d_%s_val" % (n, f)])) / float(ref["merged_%d_%s_max" % (n, f)])
            ss = abs(float(np.dot(a, a)) / float(ref["merged_%d_%s_ss" % (n, f)]) - 1.0)
            print("step", n, f, "sampled elementwise %.1e, sum of squares %.1e" % (ee, ss), flush=True)
            assert ee < ELEM_TOL[precision] and ss < 10 * ELEM_TOL[precision], (n, f, ee, ss)
    st = g.stats()
    g.close()
    print(st, flush=True)
    assert st["flags"] == 0, st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuned_run_matches_oracle(precision, monkeypatch):
    """lp_options.autotune: lp_setup times the band factorisation variants,
    the solve prefetch depths and (LP_AUTO, both paths set up) one batch of
    local Oseen solves by the band path and by the Krylov path on the run's
    own systems, keeps the fastest, and the run still matches the oracle."""
    monkeypatch.setenv("LP_KRYLOV_STRIP", "6")
    cfg = W.config("cfg1")
    g = run_parity(cfg, precision, 3, autotune=True, max_ir=4, keep=True)
    st = g.stats()
    g.close()
    print(st, flush=True)
    assert st["tuned"] == 1 and st["tune_dense_ms"] > 0 and st["tune_krylov_ms"] > 0, st
    assert st["lu_variant"] in (0, 8, 9) and st["solve_depth"] in (16, 32, 64), st
    assert (st["solver"] == 2) == (st["tune_krylov_ms"] < st["tune_dense_ms"]), st


def test_refinement_failure_is_sticky_and_reported():
    """A refinement that cannot reach its tolerance (one FP32 sweep against
    1e-14) raises flag bit 0, lp_get_stats returns LP_ERR_NOCONV with the
    statistics filled in, and the run-long maxima cover every step; a run
    that converges has no flag and maxima within the tolerance."""
    from ctypes import byref
    from paper_2311_05170_amd import lib
    g = _gpu(W.small(), "mixed", max_ir=1, ir_tol=1e-14)
    for _ in range(2):
        g.step()
    s = lib.LpStats()
    assert lib._LIB.lp_get_stats(g._h, byref(s)) == lib.LP_ERR_NOCONV
    assert s.flags & 1 and s.ir_sweeps_max == 1 and s.ir_relres_max > 1e-14, g.stats()
    g.close()
    g = _gpu(W.small(), "mixed", max_ir=6)
    for _ in range(3):
        g.step()
    st = g.stats()
    g.close()
    assert st["flags"] == 0, st
    assert 1 <= st["ir_sweeps"] <= st["ir_sweeps_max"] <= 6, st
    assert st["ir_relres"] <= st["ir_relres_max"] <= 1e-10, st


def test_index_map_matches_plan_query():
    """lp_get_index_map reads the context's own plan: the same tables as the
    host-only lp_plan_query (here with explicit shifted cuts)."""
    from paper_2311_05170_amd import lib
    cfg = W.shifted_small()
    flat = W.flat_cuts(cfg["cuts"])
    g = _gpu(cfg, "fp64")
    args = (cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"])
    for which, sub in ((0, 0), (5, 0), (1, -1), (2, -1), (3, -1), (4, -1), (3, 5), (4, 20)):
        assert np.array_equal(g.index_map(which, sub), lib.plan_query(*args, which, sub, cuts=flat)), (which, sub)
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_cfg2_timed_configuration(precision):
    """cfg2 in the configuration that bench.py times: two refinement sweeps
    launched in the mixed path, the coarse Jacobian formed every third step,
    at most ten chord steps."""
    cfg = W.config("cfg2")
    run_parity(cfg, precision, 2, max_ir=2, jacobian_every=3, max_newton=10)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg2_pipeline_matches_serial(precision, monkeypatch):
    """At full size, 12 steps issued back to back (every ring wraps) give
    bit-identical fields to the serial schedule, with no flag raised."""
    cfg = W.config("cfg2")
    kw = dict(max_ir=2, jacobian_every=3, max_newton=10)
    g = _gpu(cfg, precision, **kw)
    for _ in range(12):
        g.step()
    a = _fields(g)
    st = g.stats()
    g.close()
    assert st["flags"] == 0, st
    monkeypatch.setenv("LP_SERIAL", "1")
    g = _gpu(cfg, precision, **kw)
    for _ in range(12):
        g.step()
    b = _fields(g)
    g.close()
    for f in a:
        assert np.array_equal(a[f], b[f]), f


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_jacobian_reuse(precision):
    """The coarse Jacobian formed every third step and reused in between
    (chord steps to the same tolerance) agrees with the oracle too."""
    cfg = W.config("cfg1")
    run_parity(cfg, precision, cfg["steps"], jacobian_every=3)


def test_stokes_mode_parity():
    """Convection switched off (Stokes conduit) agrees too."""
    run_parity(W.small(), "fp64", 2, convection=False)


def test_state_machine_errors():
    from paper_2311_05170_amd.lib import LpError
    g = _gpu(W.small(), "fp64")
    with pytest.raises(LpError) as e:
        g.local_step()
    assert e.value.status == 2
    g.coarse_step()
    with pytest.raises(LpError) as e:
        g.coarse_step()
    assert e.value.status == 2
    g.local_step()
    with pytest.raises(LpError):
        g.solution("u", "local", sub=0)        # porous subdomain has no velocity
    g.close()


def test_newton_cap_sets_sticky_flag():
    """A coarse step that reaches the iteration cap unconverged raises flag bit
    1, and the flag stays set after later steps (one chord step cannot reach
    1e-13 from the extrapolated start)."""
    g = _gpu(W.small(), "fp64", max_newton=1)
    g.step()
    g.step()
    assert g.stats()["flags"] & 2
    g.close()
    g = _gpu(W.small(), "fp64")
    for _ in range(3):
        g.step()
    st = g.stats()
    assert st["flags"] == 0 and 1 <= st["newton_its"] <= st["newton_its_max"] <= 16, st
    g.close()


RAGGED_PRM = dict(W.unit_params(), nu=0.05, k=[0.3, 0.02, 0.004], sigma=2.0, sigma_star=0.5)


def _ragged():
    return W.small(NH=3, refine=4, nsub=3, overlap=1, dt=0.02, prm=RAGGED_PRM)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("variant", ["0", "8", "9"])
def test_parity_lu_kernels(precision, variant, monkeypatch):
    """Every band factorisation (variant 0: elimination on the vector units;
    8: blocked, trailing updates on the matrix cores; 9: the blocked one with
    a one-panel lookahead, FP32 factors only) for every system of the run
    (porous, coarse and local Oseen) agrees with the oracle."""
    monkeypatch.setenv("LP_LU_VARIANT", variant)
    run_parity(_ragged(), precision, 3)


@pytest.mark.parametrize("depth", ["16", "32", "64"])
def test_parity_solve_prefetch_depths(depth, monkeypatch):
    """The band solves with 16, 32 or 64 factor columns in flight (64: FP32
    only, the FP64 solves then take 32) agree with the oracle."""
    monkeypatch.setenv("LP_SOLVE_DEPTH", depth)
    run_parity(_ragged(), "mixed", 2)


def _fields(g):
    return {f: g.solution(f) for f in ("u", "p", "pF", "pf", "pm")}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_streams_do_not_change_results(precision, monkeypatch):
    """The overlapped schedule (coarse steps ahead of the local stage, porous
    and factor streams) gives bit-identical fields to running every stage on
    one stream in program order: no race, no order-dependent arithmetic."""
    cfg = W.config("cfg1")
    g = _gpu(cfg, precision)
    for _ in range(3):
        g.step()
    a = _fields(g)
    g.close()
    monkeypatch.setenv("LP_SERIAL", "1")
    g = _gpu(cfg, precision)
    for _ in range(3):
        g.step()
    b = _fields(g)
    g.close()
    for f in a:
        assert np.array_equal(a[f], b[f]), f


RING_STEPS = 18


@functools.lru_cache(maxsize=1)
def _oracle_after(name, steps):
    cfg = W.config(name)
    o = _oracle(cfg)
    for _ in range(steps):
        o.coarse_step()
        o.local_step()
    return o


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pipeline_wraps_its_rings(precision, monkeypatch):
    """18 steps issued back to back, with no host synchronisation between them:
    the coarse trajectory runs ahead, and the rings of coarse states and
    prolongations (8 slots) and of factor slots (5) wrap twice or more.  The
    fields are bit-identical to the serial schedule's and agree with the
    oracle after the last step (coarse Jacobian every third step, as timed)."""
    cfg = W.config("cfg1")
    kw = dict(jacobian_every=3, max_newton=10)
    g = _gpu(cfg, precision, **kw)
    for _ in range(RING_STEPS):
        g.step()
    a = _fields(g)
    o = _oracle_after("cfg1", RING_STEPS)
    em = compare(o, g, "merged")
    st = g.stats()
    g.close()
    print("after", RING_STEPS, "steps", {k: "%.1e" % v for k, v in em.items()}, st, flush=True)
    assert max(em.values()) < TOL[precision], em
    assert st["flags"] == 0, st
    monkeypatch.setenv("LP_SERIAL", "1")
    g = _gpu(cfg, precision, **kw)
    for _ in range(RING_STEPS):
        g.step()
    b = _fields(g)
    g.close()
    for f in a:
        assert np.array_equal(a[f], b[f]), f


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("solver", ["dense", "krylov"])
def test_graphs_match_serial(precision, solver, monkeypatch):
    """Graph mode (each step's launch sequences captured and replayed as HIP
    graphs, the instantiated graphs updated with each step's arguments; eight
    graphs per sequence in rotation) over 18 steps issued back to back gives
    bit-identical fields to the serial schedule without graphs, agrees with
    the oracle after the last step, and a stage-timed step in between (run
    without graphs) changes nothing."""
    cfg = W.config("cfg1")
    kw = dict(jacobian_every=3, max_newton=10, solver=solver, max_ir=4)
    if solver == "krylov":
        monkeypatch.setenv("LP_KRYLOV_STRIP", "6")
    g = _gpu(cfg, precision, graphs=True, **kw)
    for n in range(RING_STEPS):
        if n == 9:
            g.set_timing(["ose_solve"])
        g.step()
        if n == 9:
            g.timing()
            g.set_timing([])
    a = _fields(g)
    o = _oracle_after("cfg1", RING_STEPS)
    em = compare(o, g, "merged")
    st = g.stats()
    g.close()
    assert max(em.values()) < TOL[precision], em
    assert st["flags"] == 0, st
    monkeypatch.setenv("LP_SERIAL", "1")
    g = _gpu(cfg, precision, **kw)
    for _ in range(RING_STEPS):
        g.step()
    b = _fields(g)
    g.close()
    for f in a:
        assert np.array_equal(a[f], b[f]), f


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg2_graphs_match_serial(precision, monkeypatch):
    """cfg2 in the timed configuration with graphs: 12 steps bit-identical to
    the serial schedule."""
    cfg = W.config("cfg2")
    kw = dict(max_ir=2, jacobian_every=3, max_newton=10)
    g = _gpu(cfg, precision, graphs=True, **kw)
    for _ in range(12):
        g.step()
    a = _fields(g)
    st = g.stats()
    g.close()
    assert st["flags"] == 0, st
    monkeypatch.setenv("LP_SERIAL", "1")
    g = _gpu(cfg, precision, **kw)
    for _ in range(12):
        g.step()
    b = _fields(g)
    g.close()
    for f in a:
        assert np.array_equal(a[f], b[f]), f


def test_h_equals_H_gives_zero_corrections():
    """With T_h = T_H the local residual equations have zero data (every test
    function is supported inside Omega_j), so every correction vanishes and the
    merged field equals the coarse one."""
    cfg = W.small(NH=8, refine=1, nsub=4, overlap=1, dt=0.05)
    g = _gpu(cfg, "fp64")
    for _ in range(2):
        g.step()
    nsub = 2 * cfg["nsub"][0] * cfg["nsub"][1]
    for sub in range(nsub):
        fields = ("pF", "pf", "pm") if sub < nsub // 2 else ("u", "p")
        for f in fields:
            assert np.max(np.abs(g.solution(f, "local", sub))) < 1e-10, (sub, f)
    for f in ("u", "p", "pF", "pf", "pm"):
        assert np.max(np.abs(g.solution(f) - g.solution(f, "coarse"))) < 1e-10, f
    g.close()


def test_unsupported_bandwidth_is_reported():
    """The h = 1/256 workload's local Oseen systems (half-bandwidths to 399)
    do not fit the band window: with the band factorisation requested
    (LP_DENSE) lp_setup refuses them with LP_ERR_UNSUPPORTED instead of
    running out of the kernels' window."""
    from paper_2311_05170_amd.lib import LpError
    with pytest.raises(LpError) as e:
        _gpu(W.config("cfg3"), "mixed", solver="dense")
    assert e.value.status == 6
    assert "bandwidth" in str(e.value)
