"""The library's host-only planning and reference-data code (plan.cpp: the
partition of Algorithm 3 Step 2, band numbering, owner tables, Krylov strips;
fe.cpp: reference-element tables, exact nodal values, source loads) built
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer (no recovery:
any finding aborts), run over the workloads' partitions, ragged ones and
invalid cut lists.  Its sizes must also agree with the hipcc-built library's
plan tables.  CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2311_05170_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_05170_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("san")
    exe = str(out / "host_sanitize_driver")
    flags = ["-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
             "-I" + CSRC, "-I/opt/rocm/include", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    srcs = [os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), os.path.join(CSRC, "plan.cpp"),
            os.path.join(CSRC, "fe.cpp")]
    r = subprocess.run(["g++"] + flags + srcs + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, NH, refine, nsub, overlap, width, cuts=None):
    args = [exe, str(NH), str(refine), str(nsub[0]), str(nsub[1]), str(overlap), str(width)]
    args += [str(c) for c in (cuts or [])]
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run(args, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, \
        (args, r.returncode, r.stderr[-3000:])
    return r.stdout.splitlines()[-1].split()     # the last line: "ok ..." or "rejected ..."


CASES = [("cfg1", 16), ("cfg2", 16), ("cfg3", 16), ("shifted_small", 6)]


@pytest.mark.parametrize("name,width", CASES)
def test_workload_plans_are_clean(driver, name, width):
    from paper_2311_05170_amd import lib
    cfg = W.shifted_small() if name == "shifted_small" else W.config(name)
    flat = W.flat_cuts(cfg["cuts"])
    out = _run(driver, cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], width, flat)
    assert out[0] == "ok", out
    npor, nose, ldofs, maxbw = int(out[1]), int(out[2]), int(out[3]), int(out[4])
    # the same plan as the library's own build
    sizes = lib.plan_query(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], 5, cuts=flat).reshape(-1, 2)
    n = cfg["nsub"][0] * cfg["nsub"][1]
    assert npor == n and nose == n and len(sizes) == 2 * n
    assert ldofs == int(3 * sizes[:n, 0].sum() + sizes[n:, 0].sum())
    assert maxbw == int(sizes[:, 1].max())


@pytest.mark.parametrize("NH,refine,nsub,overlap", [(3, 3, (2, 2), 1), (2, 5, (3, 2), 2), (1, 7, (1, 1), 0),
                                                     (5, 2, (4, 3), 3), (2, 2, (4, 4), 1)])
def test_ragged_plans_are_clean(driver, NH, refine, nsub, overlap):
    out = _run(driver, NH, refine, nsub, overlap, 4)
    assert out[0] in ("ok", "rejected"), out


def test_invalid_cuts_are_rejected_cleanly(driver):
    N = 8
    good = [0, 4, 8]
    bad_lists = [[0, 5, 4, 8], [1, 4, 8], [0, 4, 9], [0, 4, 4, 8], [0, -3, 8]]
    for bad in bad_lists:
        if len(bad) != 3:
            continue        # a list of the wrong length is the caller's buffer: not sent
        for pos in range(4):
            lists = [good] * 4
            lists[pos] = bad
            out = _run(driver, 2, 4, (2, 2), 1, 0, [v for l in lists for v in l])
            assert out[0] == "rejected", (pos, bad, out)
    out = _run(driver, 0, 4, (2, 2), 1, 0)
    assert out[0] == "rejected"
    out = _run(driver, 2, 4, (0, 2), 1, 0)
    assert out[0] == "rejected"
    out = _run(driver, 2, 4, (2, 2), -1, 0)
    assert out[0] == "rejected"
