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


def test_library_exports_header_symbols():
    names = header_functions()
    assert set(names) == set(lib.EXPORTS)
    so = ctypes.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(so, n), n


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
    for sd in subs[:: max(1, len(subs) // 24)]:
        row = tab[sd.sid]
        assert tuple(row[:5]) == (sd.region, sd.x0, sd.x1, sd.y0, sd.y1)
        assert tuple(row[5:]) == tuple(sd.d)
        mesh = mp if sd.region == POROUS else mc
        cls = sd.classify_p2(mesh)
        assert np.array_equal(lib.plan_query(*args, 1, sd.sid, cuts=flat), cls)
        _, I, J = sd.p1_nodes(mesh)
        art = sd.artificial_p1(I, J)
        assert np.array_equal(lib.plan_query(*args, 2, sd.sid, cuts=flat), 2 * art)
        dof = lib.plan_query(*args, 3, sd.sid, cuts=flat)
        nfree = (cls == 0).sum()
        if sd.region == POROUS:
            assert sizes[sd.sid, 0] == nfree
            assert np.array_equal(np.sort(dof[dof >= 0]), np.arange(nfree))
        else:
            dp = lib.plan_query(*args, 4, sd.sid, cuts=flat)
            assert sizes[sd.sid, 0] == 2 * nfree + (~art).sum()
            allu = np.concatenate([dof[dof >= 0], dof[dof >= 0] + 1, dp[dp >= 0]])
            assert np.array_equal(np.sort(allu), np.arange(sizes[sd.sid, 0]))


def test_plan_query_rejects_bad_input():
    with pytest.raises(lib.LpError) as e:
        lib.plan_query(4, 4, (3, 3), 1, 0)            # 16 fine cells not divisible by 3
    assert e.value.status == 1
    with pytest.raises(lib.LpError):
        lib.plan_query(4, 4, (2, 2), 1, 0, cuts=[0, 9, 16] * 2 + [0, 16, 8] + [0, 8, 16])
    with pytest.raises(lib.LpError):
        lib.plan_query(4, 4, (2, 2), 1, 7)
