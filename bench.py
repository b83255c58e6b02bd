#!/usr/bin/env python
"""Throughput of the local parallel step on one MI355X.

One step = one pass of the whole per-time-step path: the FP64 coarse step
(Algorithm 3 Step 1) and the local stage (prolongation, local right-hand
sides, local porous and Oseen solves with refinement, partition-of-unity
merge; Steps 3-4).  The workload is the 2D mixed-vs-FP64 configuration
(H = 1/8, h = 1/64, 8 x 8 porous + 8 x 8 conduit subdomains, overlap 1/16,
dt = 0.01, seeded parameters).  Inputs are resident in HBM before timing.

Prints ONE JSON line.  Fields beyond the driver's contract:
  fp64            the plain FP64 GPU path on the same workload
  stages_ms       per-step stage split from a separate instrumented pass
  accuracy        max relative mass-norm error vs the CPU oracle after 2 steps
  roofline        dominant kernel (the local Oseen band factorisation)
  cpu_baseline    the CPU oracle on the host (2 steps of the same workload)
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine-grid local DoFs solved/s per time step, mixed vs FP64 at 1e-7 rel L2"
WORKLOAD = "cfg2"
PEAK_MFMA_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix peak (the factorisation's trailing updates run on MFMA)
CPU_STEPS = 2
# the instantiation the launcher picks for half-bandwidths 129..160 in FP32
LU_KERNEL = "k_band_lu_la<float,11> (local Oseen blocked band LU with one-panel lookahead, FP32, MFMA 16x16x4)"
LU_NAME = "k_band_lu_la<float,11>"


def band_lu_flops(sizes):
    """Flops of banded LU without pivoting: for column k with m = min(bw, n-1-k)
    entries below and right of the pivot: m divisions + 2 m^2 update flops."""
    tot = 0
    for n, bw in sizes:
        n, bw = int(n), int(bw)
        for k in range(n):
            m = min(bw, n - 1 - k)
            tot += m + 2 * m * m
    return tot


# Coarse chord iterations are launched up to this cap and skip themselves once
# converged; with the Jacobian formed every JACOBIAN_EVERY steps they take at
# most eight on this workload, and a step that hits the cap unconverged sets
# bit 1 of the reported flags.
MAX_NEWTON = 10
JACOBIAN_EVERY = 3
# refinement sweeps launched per local step in the mixed path (each skips once
# its system has converged; two reach the 1e-10 tolerance on this workload)
MAX_IR_MIXED = 2


def make(cfg, precision, max_ir):
    from paper_2311_05170_amd import workloads as W
    from paper_2311_05170_amd.lib import LocalParallel
    return LocalParallel(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], cfg["prm"], cfg["dt"],
                         cuts=W.flat_cuts(cfg["cuts"]), precision=precision, max_ir=max_ir,
                         max_newton=MAX_NEWTON, jacobian_every=JACOBIAN_EVERY)


def timed_run(cfg, precision, steps, warmup, max_ir):
    import torch
    from paper_2311_05170_amd import lib
    g = make(cfg, precision, max_ir)
    for _ in range(warmup):
        g.step()
    torch.cuda.synchronize()
    # timed region: only the dominant kernel is bracketed by HIP events, recorded
    # on the stream it is launched on
    g.set_timing(["ose_lu"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = g.timing()
    st = g.stats()
    lu_ms, lu_n = tm["ose_lu"]
    res = dict(ms_per_step=(t1 - t0) * 1e3 / steps, lu_ms_avg=lu_ms / max(lu_n, 1), lu_launches=lu_n, stats=st)
    # separate instrumented pass for the stage split (not part of the timed value;
    # the events serialise nothing but add launch gaps).  A few steps issued
    # first let the coarse trajectory run ahead again, so that the split is the
    # steady state's, not the refill's.
    for _ in range(4):
        g.step()
    g.set_timing(lib.STAGES)
    nd = 10
    for _ in range(nd):
        g.step()
    tm = g.timing()
    res["stages_ms"] = {k: round(v[0] / nd, 4) for k, v in tm.items()}
    g.close()
    return res


def cpu_leg(out_path):
    """Time the oracle on the host (single thread) over CPU_STEPS steps of the
    workload and store its merged fields."""
    import numpy as np
    from oracle.scheme import Oracle2D
    from paper_2311_05170_amd import workloads as W
    cfg = W.config(WORKLOAD)
    o = Oracle2D(cfg["NH"], cfg["Nh"], cfg["cuts"], cfg["overlap"], cfg["prm"], cfg["dt"])
    o.init()
    t0 = time.perf_counter()
    for _ in range(CPU_STEPS):
        o.coarse_step()
        o.local_step()
    t1 = time.perf_counter()
    m = o.merged()
    np.savez(out_path, seconds=t1 - t0, **m)


def accuracy(cfg, ref_path):
    import numpy as np
    from oracle.norms import mass_norm
    from oracle.mesh import RegionMesh
    ref = np.load(ref_path)
    mp, mc = RegionMesh(cfg["Nh"], 0), RegionMesh(cfg["Nh"], 1)
    out = {}
    for precision in ("mixed", "fp64"):
        g = make(cfg, precision, MAX_IR_MIXED if precision == "mixed" else 2)
        for _ in range(CPU_STEPS):
            g.step()
        errs = {}
        for f in ("pF", "pf", "pm", "u", "p"):
            a, b = g.solution(f), ref[f]
            mesh = mp if f in ("pF", "pf", "pm") else mc
            deg = 1 if f == "p" else 2
            nc = 2 if f == "u" else 1
            n = len(b) // nc
            num = sum(mass_norm(mesh, a[i * n:(i + 1) * n] - b[i * n:(i + 1) * n], deg) ** 2 for i in range(nc))
            den = sum(mass_norm(mesh, b[i * n:(i + 1) * n], deg) ** 2 for i in range(nc))
            errs[f] = float(np.sqrt(num / den))
        g.close()
        out[precision] = errs
    return out


def calibrate_copy(n=1 << 26, reps=3):
    """A device-to-device copy of n FP32 values (reads and writes 4 n bytes per
    launch): the yardstick that converts the FETCH_SIZE / WRITE_SIZE counters
    into HBM bytes."""
    import torch
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": reps}), flush=True)


def kernel_sha():
    """Hash of the roofline kernel's source: the row broadcast and diagonal-tile
    elimination helpers and the matrix-core traits through the end of the
    lookahead factorisation, with the barrier and broadcast helpers it calls (a
    change anywhere else in the file leaves it alone)."""
    src = open(os.path.join(ROOT, "paper_2311_05170_amd", "csrc", "kernels.hip")).read()
    a = src.index("template <int J>\n__device__ __forceinline__ float row_bcast(")
    b = src.index("void k_band_lu_la(")
    b = src.index("\n}\n", b) + 3
    parts = [src[a:b]]
    for name in ("void lds_barrier()", "T wave_bcast("):
        i = src.index(name)
        parts.append(src[src.rindex("\n", 0, i):src.index("\n}\n", i) + 3])
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


def traffic_for(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current source of the kernel."""
    path = os.path.join(ROOT, "profiles", "band_lu_cfg2_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    sha = kernel_sha()
    for line in open(path):
        if line.startswith("|") and kernel in line and workload in line and sha in line:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            try:
                return float(cells[-1])
            except ValueError:
                return None
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-leg", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration)")
    args = ap.parse_args()
    if args.cpu_leg:
        cpu_leg(args.cpu_leg)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the local stage needs no communication while "
              "time stepping and this build measures one GPU's share; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2311_05170_amd import workloads as W
    from paper_2311_05170_amd import lib
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    cfg = W.config(WORKLOAD)
    if args.warmup + args.steps + 3 > cfg["steps"]:
        print("warmup + steps + 3 exceeds the workload's %d time steps" % cfg["steps"], file=sys.stderr)
        sys.exit(2)
    flat = W.flat_cuts(cfg["cuts"])
    sizes = lib.plan_query(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], 5, cuts=flat).reshape(-1, 2)
    npor = cfg["nsub"][0] * cfg["nsub"][1]
    L = int(3 * sizes[:npor, 0].sum() + sizes[npor:, 0].sum())
    lu_flops = band_lu_flops(sizes[npor:])

    mixed = timed_run(cfg, "mixed", args.steps, args.warmup, MAX_IR_MIXED)
    fp64 = timed_run(cfg, "fp64", args.steps, args.warmup, 2)

    def rate(ms):
        return L / (ms * 1e-3)

    achieved = lu_flops / (mixed["lu_ms_avg"] * 1e-3) / 1e12     # algorithmic flops (unblocked count)
    line = {
        "metric": METRIC,
        "value": rate(mixed["ms_per_step"]),
        "unit": "local DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "2D Example-1 MMS, H=1/8, h=1/64, 8x8 porous + 8x8 conduit subdomains, "
                               "overlap 1/16, dt=0.01, SplitMix64 seed 2 parameters (cfg2)",
                   "local_dofs_per_step": L, "subdomains": int(len(sizes)),
                   "max_halfbandwidth": int(sizes[:, 1].max())},
        "fp64": {"value": rate(fp64["ms_per_step"]), "ms_per_step": fp64["ms_per_step"], "dtype": "f64"},
        "stages_ms": {"mixed": mixed["stages_ms"], "fp64": fp64["stages_ms"]},
        "refinement": {"mixed_sweeps": mixed["stats"]["ir_sweeps"], "mixed_max_sweeps": MAX_IR_MIXED,
                       "mixed_relres": mixed["stats"]["ir_relres"],
                       "fp64_relres": fp64["stats"]["ir_relres"], "flags": [mixed["stats"]["flags"], fp64["stats"]["flags"]],
                       "newton_its_max": [mixed["stats"]["newton_its_max"], fp64["stats"]["newton_its_max"]],
                       "max_newton": MAX_NEWTON, "jacobian_every": JACOBIAN_EVERY},
        "roofline": {"kernel": LU_KERNEL,
                     "bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_MFMA_FP32_TFLOPS, "traffic": traffic_for(LU_NAME, WORKLOAD),
                     "flops_per_launch": lu_flops, "avg_launch_ms": mixed["lu_ms_avg"],
                     "launches": mixed["lu_launches"]},
    }
    if not args.no_cpu:
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            ref = os.path.join(td, "oracle.npz")
            env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
            subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", ref], check=True, env=env)
            import numpy as np
            secs = float(np.load(ref)["seconds"])
            line["cpu_baseline"] = {"value": L * CPU_STEPS / secs, "unit": "local DoF/s", "cores": 1,
                                    "kind": "oracle",
                                    "sample": "%d full steps (coarse + local) of the same workload, "
                                              "NumPy/SciPy FP64, one thread, %.1f s" % (CPU_STEPS, secs)}
            line["accuracy"] = accuracy(cfg, ref)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
