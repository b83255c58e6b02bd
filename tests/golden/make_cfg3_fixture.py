"""Write a sampled record of the oracle's fields on the uneven h = 1/256
workload (H = 1/16, 16 x 16 + 16 x 16 subdomains with SplitMix64-shifted cuts,
overlap 8h, dt = 1e-3, seed 3 parameters).

Runs the FP64 CPU oracle (Algorithm 3, Steps 1-4) for 2 time steps.  The
local solves of a step (Step 3) are independent per subdomain, so they run in
a pool of forked processes; the coarse step and the merge stay in this
process.  Stored per step and merged field: every 29th entry with its index,
the largest magnitude and the sum of squares of the whole field; the coarse
fields after each step in full.  Only the oracle and the seeded workload
module are called.

    python tests/golden/make_cfg3_fixture.py      (a few minutes on 8 cores)
"""
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.mesh import POROUS  # noqa: E402
from oracle.scheme import Oracle2D  # noqa: E402
from paper_2311_05170_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "cfg3_oracle_sampled.npz")
STEPS = 2
STRIDE = 29
_STATE = {}


def _solve(sid):
    o, pro = _STATE["o"], _STATE["pro"]
    sd = o.subs[sid]
    return sid, (o.local_porous(sd, pro) if sd.region == POROUS else o.local_conduit(sd, pro))


def main():
    cfg = W.config("cfg3")
    o = Oracle2D(cfg["NH"], cfg["Nh"], cfg["cuts"], cfg["overlap"], cfg["prm"], cfg["dt"])
    o.init()
    out = {"stride": np.array(STRIDE)}
    ctx = mp.get_context("fork")
    for n in range(1, STEPS + 1):
        o.coarse_step()
        pro = o.prolonged()
        _STATE["o"], _STATE["pro"] = o, pro
        with ctx.Pool(min(8, os.cpu_count() or 1)) as pool:
            res = pool.map(_solve, [sd.sid for sd in o.subs], chunksize=4)
        o.e = dict(res)
        o.n += 1
        o._pro = pro
        for f, v in o.merged().items():
            out["merged_%d_%s_val" % (n, f)] = v[::STRIDE].copy()
            out["merged_%d_%s_max" % (n, f)] = np.array(np.max(np.abs(v)))
            out["merged_%d_%s_ss" % (n, f)] = np.array(float(np.dot(v, v)))
        for f, v in o.coarse().items():
            out["coarse_%d_%s" % (n, f)] = v
        print("step", n, flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
