"""Write the oracle's cfg2 fields over the window that bench.py times.

Runs the FP64 CPU oracle (Algorithm 3, Steps 1-4) on the 2D mixed-vs-FP64
workload (H = 1/8, h = 1/64, 8 x 8 + 8 x 8 subdomains, overlap 1/16,
dt = 0.01, SplitMix64 seed 2 parameters) for 25 time steps and stores the
merged fine fields after steps 12 and 25 and the coarse fields after step 25.
Only the oracle and the seeded workload module are called.

    python tests/golden/make_cfg2_fixture.py      (about a minute)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.scheme import Oracle2D  # noqa: E402
from paper_2311_05170_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "cfg2_oracle_steps.npz")
STEPS = (12, 25)


def main():
    cfg = W.config("cfg2")
    o = Oracle2D(cfg["NH"], cfg["Nh"], cfg["cuts"], cfg["overlap"], cfg["prm"], cfg["dt"])
    o.init()
    out = {}
    for n in range(1, max(STEPS) + 1):
        o.coarse_step()
        o.local_step()
        if n in STEPS:
            for f, v in o.merged().items():
                out["merged_%d_%s" % (n, f)] = v
            print("step", n, flush=True)
    for f, v in o.coarse().items():
        out["coarse_%d_%s" % (max(STEPS), f)] = v
    np.savez_compressed(OUT, steps=np.array(STEPS), **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
