"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-side partition tables equal the oracle's bit for
bit (subdomain boxes, node classes, unknown counts)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.mesh import RegionMesh, make_subdomains, POROUS
from paper_2311_05170_amd import lib, workloads as W

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lp.h")


def header_functions():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"\b(lp_[a-z_]+)\s*\(", txt)))


def header_prototypes():
    """{function name: parameter count} of every prototype in lp.h."""
    txt = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b(lp_[a-z_]+)\s*\(([^)]*)\)\s*;", txt):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else len(args.split(","))
    return out


def test_library_exports_header_symbols():
    names = header_functions()
    assert set(names) == set(lib.EXPORTS)
    so = ctypes.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(so, n), n


def test_binding_signatures_match_header():
    """Every prototype of lp.h has as many parameters as the binding passes
    (lp_setup takes the samples array, lp_get_solution the sample index)."""
    protos = header_prototypes()
    assert set(protos) == set(lib.EXPORTS)
    for name, nargs in protos.items():
        fn = getattr(lib._LIB, name)
        if fn.argtypes is not None:
            assert len(fn.argtypes) == nargs, (name, len(fn.argtypes), nargs)
    assert protos["lp_get_solution"] == 9 and protos["lp_get_index_map"] == 6
    txt = open(HDR).read()
    assert "const lp_params *samples" in txt
    for field in ("solver", "coarse_ns", "krylov_tol", "max_iter", "nsamples"):
        assert field in dict(lib.LpOptions._fields_), field
    for field in ("ir_sweeps_max", "ir_relres_max"):
        assert field in dict(lib.LpStats._fields_), field


def _struct_fields(name):
    """Field names of a typedef struct of lp.h, in declaration order."""
    txt = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", txt)
    assert m, name
    out = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(","):
            nm = re.sub(r"\[.*?\]", "", part).split()[-1].lstrip("*")
            out.append(nm)
    return out


@pytest.mark.parametrize("cname,pyname", [("lp_stats", "LpStats"), ("lp_options", "LpOptions"),
                                          ("lp_params", "LpParams"), ("lp_mesh", "LpMesh")])
def test_binding_structs_match_header(cname, pyname):
    """The ctypes mirrors of the header's structs list the same fields in the
    same order (a field out of place would shift every later one)."""
    assert [f for f, _ in getattr(lib, pyname)._fields_] == _struct_fields(cname)


def _setup_status(opt_kw=None, samples=None, prm_kw=None, dts=None):
    """Call lp_setup with options that it rejects before touching a device."""
    from ctypes import byref, c_void_p
    mesh, part, keep = lib._structs(2, 4, (2, 2), 1, None)
    opt = lib.LpOptions()
    opt.problem, opt.precision, opt.convection, opt.max_ir, opt.ir_tol = 0, lib.LP_MIXED, 1, 4, 1e-10
    opt.max_newton, opt.newton_tol, opt.jacobian_every = 8, 1e-13, 1
    opt.solver, opt.coarse_ns, opt.krylov_tol, opt.max_iter, opt.nsamples = 0, 0, 1e-12, 30, 1
    for k, v in (opt_kw or {}).items():
        setattr(opt, k, v)
    plist = samples or [dict(W.unit_params(), **(prm_kw or {}))]
    dts = dts or [0.05] * len(plist)
    arr = (lib.LpParams * len(plist))(*[lib._params(q, t) for q, t in zip(plist, dts)])
    h = c_void_p()
    st = lib._LIB.lp_setup(byref(mesh), byref(part), arr, byref(opt), None, None, byref(h))
    assert not h.value
    return st, lib._LIB.lp_last_error().decode()


def test_setup_rejects_bad_options_without_a_device():
    """Argument checks run before any device call: unknown option values and
    invalid parameters (and samples with different dt) are LP_ERR_ARG, requests
    this build does not implement (several samples with the Krylov path or
    Algorithm 1; the semi-implicit coarse step)
    LP_ERR_UNSUPPORTED."""
    assert _setup_status({"solver": 7})[0] == 1
    assert _setup_status({"coarse_ns": 3})[0] == 1
    assert _setup_status({"nsamples": -1})[0] == 1
    assert _setup_status({"precision": 5})[0] == 1
    assert _setup_status({"max_ir": 0})[0] == 1
    st, msg = _setup_status(prm_kw={"nu": -1.0})
    assert st == 1 and "sample 0" in msg
    st, msg = _setup_status({"nsamples": 2}, samples=[W.unit_params(), dict(W.unit_params(), k=[0.0, 1, 1])])
    assert st == 1 and "sample 1" in msg          # every sample is validated
    st, msg = _setup_status({"nsamples": 2}, samples=[W.unit_params(), W.unit_params()], dts=[0.05, 0.02])
    assert st == 1 and "dt" in msg                # samples share one time grid
    for kw in ({"solver": lib.LP_KRYLOV}, {"scheme": lib.LP_ONE_GRID}):
        assert _setup_status(dict(kw, nsamples=2), samples=[W.unit_params()] * 2)[0] == 6, kw
    assert _setup_status({"solver": lib.LP_KRYLOV, "max_iter": 65})[0] == 1
    assert _setup_status({"solver": lib.LP_KRYLOV, "krylov_tol": 0.0})[0] == 1
    assert _setup_status({"krylov_cycles": 5})[0] == 1            # more cycles than refinement sweeps
    assert _setup_status({"coarse_ns": lib.LP_SEMI_IMPLICIT})[0] == 6
    assert _setup_status({"scheme": 2})[0] == 1
    assert _setup_status({"lagged": 2})[0] == 1
    st, msg = _setup_status({"scheme": lib.LP_ONE_GRID})          # Algorithm 1 needs refine = 1
    assert st == 1 and "refine" in msg


@pytest.mark.parametrize("name,width", [("cfg3", 16), ("cfg2", 6), ("cfg1", 5)])
def test_krylov_strips_cover_each_box(name, width):
    """The Krylov path's preconditioner strips (one query): every conduit box
    is cut along x into strips of at most `width` cells with 2 cells of
    overlap, strips span the box's height, consecutive strips overlap, and
    every strip's band fits the 159 window (the library also checks that the
    strips' owned unknowns partition each box's unknowns)."""
    cfg = W.config(name)
    flat = W.flat_cuts(cfg["cuts"])
    args = (cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"])
    tab = lib.plan_query(*args, 0, cuts=flat).reshape(-1, 9)
    st = lib.plan_query(*args, 7, width, cuts=flat).reshape(-1, 7)
    npor = cfg["nsub"][0] * cfg["nsub"][1]
    assert (st[:, 6] <= 159).all() and (st[:, 2] - st[:, 1] <= width).all()
    for j in range(len(tab) - npor):
        box = tab[npor + j]
        mine = st[st[:, 0] == j]
        assert len(mine) >= 1
        assert mine[0, 1] == box[1] and mine[-1, 2] == box[2]
        assert (mine[:, 3] == box[3]).all() and (mine[:, 4] == box[4]).all()
        assert (mine[1:, 1] < mine[:-1, 2]).all()          # neighbours overlap
        if box[2] - box[1] <= width:
            assert len(mine) == 1


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3"])
def test_partition_tables_match_oracle(name):
    cfg = W.config(name)
    flat = W.flat_cuts(cfg["cuts"])
    args = (cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"])
    tab = lib.plan_query(*args, 0, cuts=flat).reshape(-1, 9)
    subs = make_subdomains(cfg["Nh"], cfg["cuts"], cfg["overlap"])
    mp, mc = RegionMesh(cfg["Nh"], 0), RegionMesh(cfg["Nh"], 1)
    assert len(tab) == len(subs)
    sizes = lib.plan_query(*args, 5, cuts=flat).reshape(-1, 2)
    # every subdomain's tables, in id order (one query each)
    all_cls2, all_cls1, all_dof2, all_dof1 = (lib.plan_query(*args, w, -1, cuts=flat) for w in (1, 2, 3, 4))
    o2 = o1 = o1c = 0
    for sd in subs:
        row = tab[sd.sid]
        assert tuple(row[:5]) == (sd.region, sd.x0, sd.x1, sd.y0, sd.y1)
        assert tuple(row[5:]) == tuple(sd.d)
        mesh = mp if sd.region == POROUS else mc
        cls = sd.classify_p2(mesh)
        _, I, J = sd.p1_nodes(mesh)
        art = sd.artificial_p1(I, J)
        n2, n1 = len(cls), len(art)
        assert np.array_equal(all_cls2[o2:o2 + n2], cls), sd.sid
        assert np.array_equal(all_cls1[o1:o1 + n1], 2 * art), sd.sid
        dof = all_dof2[o2:o2 + n2]
        o2 += n2
        o1 += n1
        nfree = (cls == 0).sum()
        if sd.region == POROUS:
            assert sizes[sd.sid, 0] == nfree
            assert np.array_equal(np.sort(dof[dof >= 0]), np.arange(nfree))
        else:
            dp = all_dof1[o1c:o1c + n1]
            o1c += n1
            assert sizes[sd.sid, 0] == 2 * nfree + (~art).sum()
            allu = np.concatenate([dof[dof >= 0], dof[dof >= 0] + 1, dp[dp >= 0]])
            assert np.array_equal(np.sort(allu), np.arange(sizes[sd.sid, 0]))
    assert o2 == len(all_cls2) and o1 == len(all_cls1) and o1c == len(all_dof1)
    # the single-subdomain queries return the same slices
    for sd in subs[:: max(1, len(subs) // 8)]:
        assert np.array_equal(lib.plan_query(*args, 1, sd.sid, cuts=flat), sd.classify_p2(mp if sd.region == POROUS else mc))


def test_plan_query_rejects_bad_input():
    with pytest.raises(lib.LpError) as e:
        lib.plan_query(4, 4, (3, 3), 1, 0)            # 16 fine cells not divisible by 3
    assert e.value.status == 1
    with pytest.raises(lib.LpError):
        lib.plan_query(4, 4, (2, 2), 1, 0, cuts=[0, 9, 16] * 2 + [0, 16, 8] + [0, 8, 16])
    with pytest.raises(lib.LpError):
        lib.plan_query(4, 4, (2, 2), 1, 7)
