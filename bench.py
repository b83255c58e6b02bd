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
  refinement      run-long refinement and Newton statistics of the timed runs
                  (sticky flags: the run exits non-zero if any is raised)
  accuracy        relative mass-norm error vs the CPU oracle after CPU_STEPS (6) steps
  roofline        dominant kernel (the local Oseen band factorisation) against
                  its binding roof, plus whole-step roofline fractions of the
                  mixed and FP64 paths
  cpu_baseline    the CPU oracle on the host: a process pool over subdomains
                  on the host cores (and one thread), 6 steps of the workload
  ensemble        32 seeded parameter samples on the same geometry, all
                  samples' systems in every launch (lp_options.nsamples),
                  against the same samples run one context after another
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
PEAK_FP64_TFLOPS = 78.6         # MI355X FP64 vector and matrix peak
PEAK_HBM_GBS = 8000.0           # MI355X HBM3E
CPU_STEPS = 6                   # oracle steps of the CPU baseline (about 13 s on one host core)
CPU_POOL_MAX = 16               # host cores given to one GPU's share
SERIAL_STEPS = 8                # roofline pass: LU launches timed on an uncontended stream
ENSEMBLE_SAMPLES, ENSEMBLE_WARMUP, ENSEMBLE_STEPS = 32, 2, 8
# the ensemble's parameters span decades (viscosity to 1e-3, permeabilities to
# 1e-5): it runs with the library's default iteration limits, a Jacobian every
# Newton iteration
ENSEMBLE_MAX_IR = {"mixed": 8, "fp64": 4}
ENSEMBLE_MAX_NEWTON, ENSEMBLE_JACOBIAN_EVERY = 16, 1
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
# refinement sweeps launched on the uneven h = 1/256 workload: the mixed
# path's FP32 porous solves take three to the 1e-10 tolerance (the FP64 path
# one; later sweeps skip themselves); the local Oseen systems take one GMRES
# cycle (restart 30, stopping a decade below the tolerance), so one cycle is
# launched and a second for safety
UNEVEN_MAX_IR = 3
UNEVEN_KRYLOV_CYCLES = 2
UNEVEN_STEPS, UNEVEN_WARMUP = 5, 2


def make(cfg, precision, max_ir, graphs=False, lagged="own"):
    from paper_2311_05170_amd import workloads as W
    from paper_2311_05170_amd.lib import LocalParallel
    return LocalParallel(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], cfg["prm"], cfg["dt"],
                         cuts=W.flat_cuts(cfg["cuts"]), precision=precision, max_ir=max_ir,
                         max_newton=MAX_NEWTON, jacobian_every=JACOBIAN_EVERY, graphs=graphs, lagged=lagged)


def graph_run(cfg, precision, steps, warmup, max_ir):
    """The same timed region with every step's launch sequences replayed as
    HIP graphs (lp_options.graphs)."""
    import torch
    g = make(cfg, precision, max_ir, graphs=True)
    for _ in range(warmup):
        g.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = g.stats()
    g.close()
    return dict(ms_per_step=(t1 - t0) * 1e3 / steps, stats=st)


def timed_run(cfg, precision, steps, warmup, max_ir, lagged="own"):
    import torch
    from paper_2311_05170_amd import lib
    g = make(cfg, precision, max_ir, lagged=lagged)
    for _ in range(warmup):
        g.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # run-long statistics: the flags are sticky and the refinement maxima
    # cover every step so far (warmup and timed)
    st = g.stats()
    res = dict(ms_per_step=(t1 - t0) * 1e3 / steps, stats=st)
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


def uneven_run(precision, steps, warmup):
    """The uneven h = 1/256 workload (16 x 16 + 16 x 16 subdomains, shifted
    cuts, dt = 1e-3): the local Oseen systems (half-bandwidths to 399) go to
    the Krylov path, the porous ones to the band factorisation.  Returns its
    throughput, the run-long statistics and the stage split of a few
    instrumented steps."""
    import torch
    from paper_2311_05170_amd import workloads as W
    from paper_2311_05170_amd.lib import LocalParallel
    from paper_2311_05170_amd import lib
    cfg = W.config("cfg3")
    t0 = time.perf_counter()
    g = LocalParallel(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], cfg["prm"], cfg["dt"],
                      cuts=W.flat_cuts(cfg["cuts"]), precision=precision, max_ir=UNEVEN_MAX_IR,
                      krylov_cycles=UNEVEN_KRYLOV_CYCLES, max_newton=MAX_NEWTON, jacobian_every=JACOBIAN_EVERY)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    for _ in range(warmup):
        g.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    st = g.stats()
    g.set_timing(lib.STAGES)
    nd = 2
    for _ in range(nd):
        g.step()
    tm = g.timing()
    g.close()
    return dict(ms_per_step=ms, stats=st, setup_s=setup_s,
                stages_ms={k: round(v[0] / nd, 3) for k, v in tm.items() if v[1]})


def scheme_comparison(steps=20, warmup=3):
    """Algorithm 1 (one grid, lp_options.scheme = LP_ONE_GRID) against
    Algorithm 3 on the same fine grid h = 1/16 (cfg1: H = 1/4, 4 x 4 + 4 x 4
    subdomains, overlap 2h, unit parameters, dt = 0.1): wall time per step of
    each, the comparison of the paper's Tables 2 and 4 on this GPU.  Algorithm
    1 solves the global fine systems in FP64 (decoupled porous solves, then the
    Navier-Stokes step by chord iterations to newton_tol)."""
    import torch
    from paper_2311_05170_amd import workloads as W
    from paper_2311_05170_amd.lib import LocalParallel
    cfg = W.config("cfg1")
    out = {}

    def clock(g):
        for _ in range(warmup):
            g.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        st = g.stats()
        g.close()
        return ms, st

    # both schemes with the library's default nonlinear iteration (Jacobian
    # formed every step, at most 16 iterations)
    ms, st = clock(LocalParallel(cfg["Nh"], 1, cfg["nsub"], 1, cfg["prm"], cfg["dt"], precision="fp64",
                                 scheme="one_grid"))
    out["algorithm1_fp64"] = {"ms_per_step": ms, "newton_its_max": st["newton_its_max"], "flags": st["flags"]}
    for prec, max_ir in (("mixed", MAX_IR_MIXED), ("fp64", 2)):
        ms, st = clock(LocalParallel(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], cfg["prm"], cfg["dt"],
                                     cuts=W.flat_cuts(cfg["cuts"]), precision=prec, max_ir=max_ir))
        out["algorithm3_" + prec] = {"ms_per_step": ms, "newton_its_max": st["newton_its_max"], "flags": st["flags"]}
    out["workload"] = ("2D Example-1 MMS, fine h=1/16 (cfg1): Algorithm 1 on T_h against Algorithm 3 with H=1/4, "
                       "4x4 porous + 4x4 conduit subdomains, overlap 2h, unit parameters, dt=0.1")
    out["steps"], out["warmup"] = steps, warmup
    out["time_ratio_alg3_mixed_to_alg1"] = out["algorithm3_mixed"]["ms_per_step"] / out["algorithm1_fp64"]["ms_per_step"]
    return out


def serial_lu_time(cfg, precision, max_ir, steps=SERIAL_STEPS):
    """Average duration of the local Oseen factorisation with nothing beside it:
    every stage on one stream in program order (LP_SERIAL=1), HIP events
    recorded around each launch on that stream.  In the overlapped schedule the
    same kernel shares the chip with the coarse chain and the solves, so its
    event interval there also holds waiting for compute units."""
    import torch
    os.environ["LP_SERIAL"] = "1"
    try:
        g = make(cfg, precision, max_ir)
    finally:
        del os.environ["LP_SERIAL"]
    for _ in range(2):
        g.step()
    torch.cuda.synchronize()
    g.set_timing(["ose_lu"])
    for _ in range(steps):
        g.step()
    ms, n = g.timing()["ose_lu"]
    g.close()
    return ms / max(n, 1), n


def ensemble_run(L, lu_bytes, lean=False):
    """The parameter ensemble (ENSEMBLE_SAMPLES seeded samples on the cfg2
    geometry, dt = 0.01, 10 steps): one context holding every sample, so that
    each launch covers all samples' systems, against the same samples stepped
    one context after another (each context's setup outside its timed steps).
    Also the ensemble's local Oseen factorisation timed on an uncontended
    stream, as the roofline pass does for one sample.  lean: the mixed
    ensemble pass and the factorisation pass only (profiling runs)."""
    import torch
    from paper_2311_05170_amd import workloads as W
    from paper_2311_05170_amd.lib import LocalParallel
    cfg = W.ensemble(ENSEMBLE_SAMPLES)
    samples = cfg["samples"]
    S = len(samples)

    def build(plist, prec, graphs=False):
        return LocalParallel(cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"], plist[0], cfg["dt"],
                             cuts=W.flat_cuts(cfg["cuts"]), precision=prec, max_ir=ENSEMBLE_MAX_IR[prec],
                             max_newton=ENSEMBLE_MAX_NEWTON, jacobian_every=ENSEMBLE_JACOBIAN_EVERY, samples=plist,
                             graphs=graphs)

    def clock(g):
        for _ in range(ENSEMBLE_WARMUP):
            g.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(ENSEMBLE_STEPS):
            g.step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / ENSEMBLE_STEPS

    out = {"workload": "2D Example-1 MMS on the cfg2 geometry (H=1/8, h=1/64, 8x8 porous + 8x8 conduit "
                       "subdomains, overlap 1/16), dt=0.01, %d SplitMix64 seed-5 samples: nu logU[1e-3,1], "
                       "k_F, k_f, k_m logU[1e-5,1], sigma*, sigma logU[0.01,10]" % S,
           "samples": S, "steps": ENSEMBLE_STEPS, "warmup": ENSEMBLE_WARMUP,
           "max_ir": ENSEMBLE_MAX_IR, "max_newton": ENSEMBLE_MAX_NEWTON, "jacobian_every": ENSEMBLE_JACOBIAN_EVERY,
           "local_dofs_per_step": S * L}
    for prec in ("mixed",) if lean else ("mixed", "fp64"):
        t0 = time.perf_counter()
        g = build(samples, prec)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        ms = clock(g)
        st = g.stats()
        g.close()
        seq = float("nan")
        if not lean:
            seq = 0.0
            for q in samples:
                h = build([q], prec)
                seq += clock(h)
                h.close()
        out[prec] = {"value": S * L / (ms * 1e-3), "ms_per_step": ms, "setup_s": setup_s,
                     "sequential_value": S * L / (seq * 1e-3), "sequential_ms_per_step": seq,
                     "speedup_vs_sequential": seq / ms,
                     "flags": st["flags"], "newton_its_max": st["newton_its_max"],
                     "sweeps_max": st["ir_sweeps_max"], "relres_max": st["ir_relres_max"],
                     "lu_growth_local": st["lu_growth_local"], "lu_pivot_local": st["lu_pivot_local"]}
    if not lean:
        # the same timed steps with every launch sequence replayed as a HIP graph
        g = build(samples, "mixed", graphs=True)
        ms = clock(g)
        st = g.stats()
        g.close()
        out["mixed"]["graphs"] = {"value": S * L / (ms * 1e-3), "ms_per_step": ms, "flags": st["flags"]}
    os.environ["LP_SERIAL"] = "1"
    try:
        g = build(samples, "mixed")
    finally:
        del os.environ["LP_SERIAL"]
    for _ in range(2):
        g.step()
    torch.cuda.synchronize()
    g.set_timing(["ose_lu"])
    for _ in range(4):
        g.step()
    lms, n = g.timing()["ose_lu"]
    g.close()
    lms /= max(n, 1)
    gbs = S * lu_bytes / (lms * 1e-3) / 1e9
    out["lu_roofline"] = {"kernel": LU_NAME, "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": gbs / PEAK_HBM_GBS, "bytes_per_launch": S * lu_bytes, "avg_launch_ms": lms,
                          "launches": n, "systems_per_launch": S * cfg["nsub"][0] * cfg["nsub"][1],
                          "timing": "HIP events around each launch, every stage on one stream (LP_SERIAL=1)"}
    out["flags_meaning"] = ("bit 0 refinement above ir_tol, bit 1 coarse Newton above newton_tol, "
                            "bit 2 pivot monitor: a factorisation without pivoting exceeded its growth or "
                            "small-pivot limit (the refinement test still decides the result)")
    return out


def step_roofline(cfg, sizes, tab, coarse, stats, T, jacobian_every):
    """Roofline time of one step: the sum over the stages of
    max(algorithmic bytes / HBM bandwidth, algorithmic flops / peak), each input
    read once and each output written once from HBM, at the measured sweep and
    Newton counts.  T = bytes per band / factor entry (4 mixed, 8 FP64).
    Returns (milliseconds, {stage: (bytes, flops)})."""
    import numpy as np
    npor = cfg["nsub"][0] * cfg["nsub"][1]
    n = sizes[:, 0].astype(np.float64)
    bw = sizes[:, 1].astype(np.float64)
    # local lattice nodes per subdomain: (2 cx + 1)(2 cy + 1) P2, (cx + 1)(cy + 1) P1
    cx = (tab[:, 2] - tab[:, 1]).astype(np.float64)
    cy = (tab[:, 4] - tab[:, 3]).astype(np.float64)
    n2 = (2 * cx + 1) * (2 * cy + 1)
    n1 = (cx + 1) * (cy + 1)
    P, O = slice(0, npor), slice(npor, None)
    Nh, NH = cfg["Nh"], cfg["NH"]
    nf2, nf1 = (2 * Nh + 1) ** 2, (Nh + 1) ** 2
    sweeps = max(int(stats["ir_sweeps"]), 1)
    band = lambda nn, bb: nn * (2 * bb + 1) * T                   # noqa: E731
    fac = lambda nn, bb: (2 * nn * bb + nn) * T                   # noqa: E731
    lu_fl = float(band_lu_flops(sizes[O]))
    st = {}
    # Algorithm 3 Step 1 (coarse): each chord step reads the n x n inverse once;
    # a refresh step forms the band (written, read by the LU), its factors and
    # the inverse (written once)
    ncp, bcp, ncn, bcn = (float(v) for v in coarse)
    its = max(int(stats["newton_its"]), 1)
    refresh = (8.0 * ncn ** 2 + 2 * 8.0 * ncn * (2 * bcn + 1)) / max(jacobian_every, 1)
    st["coarse"] = (its * 8.0 * ncn ** 2 + 3 * 8.0 * ncp ** 2 + refresh,
                    its * 2.0 * ncn ** 2 + 3 * 2.0 * ncp ** 2 + float(band_lu_flops([(ncn, bcn)])) / max(jacobian_every, 1))
    # Pi_h: 6 + 7 fine fields written
    st["prolong"] = (8.0 * (12 * nf2 + nf1), 0.0)
    # local right-hand sides: read the prolonged fields and e^n, write b and e^{n+1}'s Dirichlet values
    st["por_rhs"] = (float((8.0 * (7 + 3 + 3 + 3) * n2[P]).sum()), 0.0)
    st["ose_rhs"] = (float((8.0 * (6 + 2 + 2 + 3) * n2[O] + 8.0 * 2 * n1[O]).sum()), 0.0)
    st["ose_asm"] = (float(band(n[O], bw[O]).sum()), 0.0)
    st["ose_lu"] = (float(band(n[O], bw[O]).sum() + fac(n[O], bw[O]).sum()), lu_fl)
    # per sweep: factors read once, r read and x updated (FP64); FP64 residual: x, b read, r written
    st["ose_solve"] = (sweeps * float((fac(n[O], bw[O]) + 24.0 * n[O]).sum()), sweeps * float((4 * n[O] * bw[O]).sum()))
    st["por_solve"] = (sweeps * float(3 * (fac(n[P], bw[P]) + 24.0 * n[P]).sum()), sweeps * float((12 * n[P] * bw[P]).sum()))
    st["ose_res"] = (sweeps * float((24.0 * n[O] + 16.0 * n2[O]).sum()), 0.0)
    st["por_res"] = (sweeps * float((3 * 24.0 * n[P]).sum()), 0.0)
    # finalize and merge: e^{n+1} written once, read by the merge with the
    # prolonged base; the merged fields written
    st["merge"] = (float(8.0 * (3 * n2[P].sum() + 2 * n2[O].sum() + n1[O].sum())) * 2 + 8.0 * 2 * (5 * nf2 + nf1), 0.0)
    peak = (PEAK_MFMA_FP32_TFLOPS if T == 4 else PEAK_FP64_TFLOPS) * 1e12
    t = sum(max(b / (PEAK_HBM_GBS * 1e9), f / peak) for b, f in st.values())
    return t * 1e3, {k: {"bytes": v[0], "flops": v[1]} for k, v in st.items()}


def cpu_leg(out_path, pool):
    """Time the oracle on the host over CPU_STEPS steps of the workload and
    store its merged fields.  pool = 1: one thread; pool > 1: each step's local
    solves (Step 3, independent per subdomain) go to `pool` forked worker
    processes, one BLAS thread each, the coarse step and the merge stay in the
    parent.  The oracle's constant local porous operators are built before the
    clock starts (the library factors them at setup as well)."""
    import multiprocessing as mp
    import numpy as np
    from oracle.mesh import POROUS
    from oracle.scheme import Oracle2D
    from paper_2311_05170_amd import workloads as W
    cfg = W.config(WORKLOAD)
    o = Oracle2D(cfg["NH"], cfg["Nh"], cfg["cuts"], cfg["overlap"], cfg["prm"], cfg["dt"])
    o.init()
    for sd in o.subs:
        if sd.region == POROUS:
            o._porous_ops(sd)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    for _ in range(CPU_STEPS):
        o.coarse_step()
        if pool <= 1:
            o.local_step()
            continue
        pro = o.prolonged()
        _POOL_STATE["o"], _POOL_STATE["pro"] = o, pro
        order = sorted(o.subs, key=lambda sd: -(sd.x1 - sd.x0) * (sd.y1 - sd.y0) * (1 if sd.region == POROUS else 3))
        with ctx.Pool(pool) as pl:
            res = pl.map(_pool_solve, [sd.sid for sd in order], chunksize=1)
        o.e = dict(res)
        o.n += 1
        o._pro = pro
    t1 = time.perf_counter()
    m = o.merged()
    np.savez(out_path, seconds=t1 - t0, **m)


_POOL_STATE = {}


def _pool_solve(sid):
    from oracle.mesh import POROUS
    o, pro = _POOL_STATE["o"], _POOL_STATE["pro"]
    sd = o.subs[sid]
    return sid, (o.local_porous(sd, pro) if sd.region == POROUS else o.local_conduit(sd, pro))


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


def summarize_trace(path, last=SERIAL_STEPS, split=False):
    """Per-kernel launch counts and average durations from a rocprofv3
    kernel-trace CSV, and for the roofline kernel the average of its last
    `last` launches (the uncontended pass that bench.py times with events)
    beside that of its earlier, overlapped ones.  split: also every kernel's
    time per step over the steps of those last launches (from the end of the
    launch before them to the end of the trace; meaningful when that pass is
    the run's last, as with --lean)."""
    import csv
    import re
    rows = list(csv.DictReader(open(path)))
    by = {}
    for r in rows:
        by.setdefault(r["Kernel_Name"], []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    print("| kernel | launches | avg us | total ms |")
    print("|---|---:|---:|---:|")
    tot = {k: sum(e - b for b, e in v) for k, v in by.items()}
    for k in sorted(by, key=lambda k: -tot[k]):
        v = by[k]
        print("| %s | %d | %.1f | %.3f |" % (k.replace("|", "/")[:110], len(v), tot[k] / len(v) / 1e3, tot[k] / 1e6))
    pat = re.compile(r"k_band_lu_la<float, ?11>")
    for k, v in by.items():
        if pat.search(k):
            v = sorted(v)
            d = [(e - b) / 1e3 for b, e in v]
            print("\nroofline kernel %s: last %d launches (LP_SERIAL pass) avg %.1f us; earlier %d launches "
                  "(overlapped schedule) avg %.1f us" % (k, last, sum(d[-last:]) / last, len(d) - last,
                                                         sum(d[:-last]) / max(len(d) - last, 1)))
            if split and len(v) > last:
                t0 = v[-last - 1][1]
                win = [(b, e, name) for name, lst in by.items() for b, e in lst if b > t0]
                tw = {}
                for b, e, name in win:
                    tw[name] = tw.get(name, 0) + (e - b)
                span = (max(e for _, e, _ in win) - min(b for b, _, _ in win)) / 1e6
                print("\nUncontended pass, per step (%d steps, %.2f ms span, %.2f ms of kernels):\n"
                      % (last, span, sum(tw.values()) / 1e6))
                print("| kernel | ms per step |")
                print("|---|---:|")
                for name in sorted(tw, key=lambda n: -tw[n]):
                    print("| %s | %.3f |" % (name.replace("|", "/")[:110], tw[name] / 1e6 / last))


def host_cores():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return avail, model


def run_cpu_leg(pool):
    import numpy as np
    import tempfile
    td = tempfile.mkdtemp()
    ref = os.path.join(td, "oracle.npz")
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", ref, "--cpu-pool", str(pool)],
                   check=True, env=env)
    return float(np.load(ref)["seconds"]), ref


# Algorithm 1 with the paper's own elements (lp_mini_*): Example 1 at h = 1/16,
# dt = h^2, T = 1, the workload of Table 2's second row
PAPER_N = 16
PAPER_CPU_STEPS = 24


def paper_elements_run():
    """Algorithm 1 with MINI in the conduit and P1 porous pressures on the
    device: wall time per step (every Newton iteration waits for its
    convergence test on the host), the paper's Table 2 workload at h = 1/16."""
    from paper_2311_05170_amd import workloads as W
    from paper_2311_05170_amd.lib import MiniAlgorithm1
    N = PAPER_N
    dt, nsteps, warm = 1.0 / N ** 2, N ** 2, 4
    g = MiniAlgorithm1(N, W.unit_params(), dt)
    try:
        g.step(warm)
        t0 = time.perf_counter()
        g.step(nsteps - warm)
        ms = (time.perf_counter() - t0) * 1e3 / (nsteps - warm)
        st = g.stats()
    finally:
        g.close()
    n1 = N + 1
    n, bw = 3 * n1 * n1 + 4 * N * N, 7 * N + 16
    # the dominant kernel: the FP64 band factorisation of the Navier-Stokes
    # system, once per step (chord iterations), timed by HIP events around
    # each launch over the whole run
    flops = band_lu_flops([(n, bw)])
    nbytes = float(n * (2 * bw + 1) * 8 + (2 * n * bw + n) * 8)
    lu_ms = st["lu_ms"] / max(st["lu_launches"], 1)
    roof_ms = max(nbytes / (PEAK_HBM_GBS * 1e9), flops / (PEAK_FP64_TFLOPS * 1e12)) * 1e3
    bound = "hbm" if nbytes / (PEAK_HBM_GBS * 1e9) >= flops / (PEAK_FP64_TFLOPS * 1e12) else "mfma"
    return {"workload": "2D Example-1 MMS with the paper's elements (MINI conduit, P1 porous), Algorithm 1 on "
                        "h=1/%d, dt=h^2=1/%d, T=1, unit parameters (Table 2, second row)" % (N, N * N),
            "ms_per_step": ms, "steps": nsteps - warm, "warmup": warm, "iterations_max": st["newton_its_max"],
            "flags": st["flags"],
            "unknowns": {"navier_stokes": n, "porous": 3 * n1 * n1, "ns_half_bandwidth": bw},
            "roofline": {"kernel": "k_band_lu_la<double,9> (Navier-Stokes band LU, one system)", "bound": bound,
                         "achieved": nbytes / (lu_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": roof_ms / lu_ms, "traffic": None, "bytes_per_launch": nbytes,
                         "flops_per_launch": flops, "avg_launch_ms": lu_ms, "launches": st["lu_launches"],
                         "timing": "HIP events around each launch"}}


EX3_N, EX3_STEPS, EX3_DT = 9, 200, 0.05
EX3_KF = [2e-2, 4e-2, 6e-2, 8e-2, 2e-1, 4e-1, 6e-1, 8e-1]


def example3_run():
    """The Example-3-type variant (lp_mini_setup with LP_EX3_2D) over the
    paper's k_F sweep: h = 1/9, dt = 0.05, T = 10 as Example 3, on the
    two-square geometry; the outflow rate through the conduit top (the P1
    trace of u_y, trapezoid) and the wall time per step."""
    from paper_2311_05170_amd.lib import MiniAlgorithm1
    N = EX3_N
    nb = (N + 1) ** 2 + 2 * N * N
    samples = [dict(phi=[1e-4, 1e-3, 1e-2], C=[1e-4] * 3, k=[kF, 1e-6, 1e-8], mu_tilde=1e-2, sigma=0.5,
                    sigma_star=0.5, rho=10.0, alpha=1.0, eta=1.0, nu=1e-2) for kF in EX3_KF]

    def run(plist):
        g = MiniAlgorithm1(N, plist[0], EX3_DT, problem="ex3", samples=plist)
        try:
            t0 = time.perf_counter()
            g.step(EX3_STEPS)
            ms = (time.perf_counter() - t0) * 1e3 / EX3_STEPS
            uys = [g.solution("u", sample=k)[nb + N * (N + 1):nb + (N + 1) ** 2] for k in range(len(plist))]
        finally:
            g.close()
        return ms, [float((uy[:-1] + uy[1:]).sum() / (2 * N)) for uy in uys]

    # the sweep as one ensemble (every launch covers the eight samples), and
    # one context per k_F, one after another
    ms_batch, rates = run(samples)
    ms_seq = sum(run([q])[0] for q in samples)
    return {"workload": "Example-3-type variant with the paper's elements: Gamma_in pressures 1.0e3/1.6e3/4.0e3, "
                        "Stokes conduit with cased walls and an outflow top, Example 3 parameters, h=1/%d, "
                        "dt=%g, T=%g" % (N, EX3_DT, EX3_STEPS * EX3_DT),
            "k_F": EX3_KF, "outflow_rate": rates, "ms_per_step_ensemble": ms_batch,
            "ms_per_step_sequential": ms_seq, "speedup": ms_seq / ms_batch}


def paper_elements_cpu():
    """The oracle's Algorithm 1 with the same elements on a bounded sample of
    the same workload (its first PAPER_CPU_STEPS steps), ms per step."""
    from paper_2311_05170_amd import workloads as W
    from oracle.mini import algorithm1_mini
    N = PAPER_N
    t0 = time.perf_counter()
    algorithm1_mini(N, W.unit_params(), 1.0 / N ** 2, PAPER_CPU_STEPS)
    return {"ms_per_step": (time.perf_counter() - t0) * 1e3 / PAPER_CPU_STEPS, "steps": PAPER_CPU_STEPS,
            "kind": "oracle", "cores": 1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-uneven", action="store_true", help="skip the h = 1/256 uneven-batch line")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the parameter-ensemble object")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="run only the parameter ensemble and print its object")
    ap.add_argument("--lean", action="store_true",
                    help="profiling runs: only the timed cfg2 passes and the roofline pass (no graphs, no scheme "
                         "comparison, no uneven line, no CPU leg)")
    ap.add_argument("--paper-only", action="store_true",
                    help="run only Algorithm 1 with the paper's elements and print its object")
    ap.add_argument("--uneven-only", action="store_true",
                    help="run only the h = 1/256 uneven batch (both precisions) and print its object")
    ap.add_argument("--cpu-leg", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-pool", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--summarize-trace", default=None, metavar="KERNEL_TRACE_CSV",
                    help="print per-kernel averages of a rocprofv3 kernel trace of this script and exit")
    ap.add_argument("--trace-last", type=int, default=SERIAL_STEPS,
                    help="with --summarize-trace: launches of the roofline kernel in the final uncontended pass")
    ap.add_argument("--trace-split", action="store_true",
                    help="with --summarize-trace: per-step kernel times of that final pass")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration)")
    args = ap.parse_args()
    if args.cpu_leg:
        cpu_leg(args.cpu_leg, args.cpu_pool)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.trace_last, args.trace_split)
        return
    if args.paper_only:
        import torch
        assert torch.cuda.is_available(), "bench.py needs a HIP device"
        out = paper_elements_run()
        out["example3"] = example3_run()
        print(json.dumps({"paper_elements": out}), flush=True)
        return
    if args.uneven_only:
        import torch
        assert torch.cuda.is_available(), "bench.py needs a HIP device"
        um = uneven_run("mixed", UNEVEN_STEPS, UNEVEN_WARMUP)
        uf = uneven_run("fp64", UNEVEN_STEPS, UNEVEN_WARMUP)
        print(json.dumps({"uneven_batch": {"mixed": {"ms_per_step": um["ms_per_step"], "stats": um["stats"]},
                                           "fp64": {"ms_per_step": uf["ms_per_step"], "stats": uf["stats"]}}}), flush=True)
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
    qargs = (cfg["NH"], cfg["refine"], cfg["nsub"], cfg["overlap"])
    sizes = lib.plan_query(*qargs, 5, cuts=flat).reshape(-1, 2)
    tab = lib.plan_query(*qargs, 0, cuts=flat).reshape(-1, 9)
    npor = cfg["nsub"][0] * cfg["nsub"][1]
    L = int(3 * sizes[:npor, 0].sum() + sizes[npor:, 0].sum())
    lu_flops = band_lu_flops(sizes[npor:])
    ose = sizes[npor:].astype(float)
    lu_bytes = float((ose[:, 0] * (2 * ose[:, 1] + 1) * 4 + (2 * ose[:, 0] * ose[:, 1] + ose[:, 0]) * 4).sum())

    if args.ensemble_only:
        print(json.dumps({"ensemble": ensemble_run(L, lu_bytes, lean=args.lean)}), flush=True)
        return
    t_start = time.perf_counter()

    def progress(what):
        print("[bench] %s done, %.1f s" % (what, time.perf_counter() - t_start), file=sys.stderr, flush=True)

    mixed = timed_run(cfg, "mixed", args.steps, args.warmup, MAX_IR_MIXED)
    progress("cfg2 mixed")
    fp64 = timed_run(cfg, "fp64", args.steps, args.warmup, 2)
    progress("cfg2 fp64")
    if args.lean:
        gmix = gf64 = None
    else:
        gmix = graph_run(cfg, "mixed", args.steps, args.warmup, MAX_IR_MIXED)
        gf64 = graph_run(cfg, "fp64", args.steps, args.warmup, 2)
        progress("cfg2 graphs")
    # the last cfg2 pass, so that its factorisations are the last launches of
    # that kernel in a kernel trace of this run (summarize_trace relies on it)
    lu_ms, lu_n = serial_lu_time(cfg, "mixed", MAX_IR_MIXED)
    progress("roofline pass")
    schemes = None if args.lean else scheme_comparison()
    if schemes:
        progress("Algorithm 1 vs 3")
    ens = None if (args.lean or args.no_ensemble) else ensemble_run(L, lu_bytes)
    if ens:
        progress("ensemble")
    # the same timed region with the lagged correction taken from the merged
    # field (lp_options.lagged = LP_LAG_MERGED): one more kernel per step
    lagm = None if args.lean else timed_run(cfg, "mixed", args.steps, args.warmup, MAX_IR_MIXED, lagged="merged")
    if lagm:
        progress("cfg2 mixed, merged lagged correction")
    paper = None if args.lean else paper_elements_run()
    if paper:
        paper["example3"] = example3_run()
        progress("paper's elements")
    uneven = None
    if not (args.no_uneven or args.lean):
        cfg3 = W.config("cfg3")
        q3 = (cfg3["NH"], cfg3["refine"], cfg3["nsub"], cfg3["overlap"])
        s3 = lib.plan_query(*q3, 5, cuts=W.flat_cuts(cfg3["cuts"])).reshape(-1, 2)
        n3 = cfg3["nsub"][0] * cfg3["nsub"][1]
        L3 = int(3 * s3[:n3, 0].sum() + s3[n3:, 0].sum())
        um = uneven_run("mixed", UNEVEN_STEPS, UNEVEN_WARMUP)
        uf = uneven_run("fp64", UNEVEN_STEPS, UNEVEN_WARMUP)
        uneven = {"workload": "2D Example-1 MMS, H=1/16, h=1/256, 16x16 porous + 16x16 conduit subdomains, "
                              "SplitMix64-shifted cuts (+-4 fine cells), overlap 8h, dt=1e-3, seed 3 parameters (cfg3)",
                  "local_dofs_per_step": L3, "steps": UNEVEN_STEPS, "warmup": UNEVEN_WARMUP,
                  "max_halfbandwidth": int(s3[:, 1].max()), "oseen_solver": "krylov",
                  "mixed": {"value": L3 / (um["ms_per_step"] * 1e-3), "ms_per_step": um["ms_per_step"],
                            "setup_s": um["setup_s"], "krylov_its": um["stats"]["krylov_its"],
                            "sweeps_max": um["stats"]["ir_sweeps_max"], "relres_max": um["stats"]["ir_relres_max"],
                            "flags": um["stats"]["flags"], "stages_ms": um["stages_ms"]},
                  "fp64": {"value": L3 / (uf["ms_per_step"] * 1e-3), "ms_per_step": uf["ms_per_step"],
                           "setup_s": uf["setup_s"], "krylov_its": uf["stats"]["krylov_its"],
                           "sweeps_max": uf["stats"]["ir_sweeps_max"], "relres_max": uf["stats"]["ir_relres_max"],
                           "flags": uf["stats"]["flags"], "stages_ms": uf["stages_ms"]}}

    def rate(ms):
        return L / (ms * 1e-3)

    # the factorisation's arithmetic intensity (flops per algorithmic byte) is
    # below the FP32 ridge (peak flops / HBM bandwidth), so HBM is its binding roof
    intensity = lu_flops / lu_bytes
    ridge = PEAK_MFMA_FP32_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    bound = "hbm" if intensity < ridge else "mfma"
    gbs = lu_bytes / (lu_ms * 1e-3) / 1e9
    tflops = lu_flops / (lu_ms * 1e-3) / 1e12
    coarse = lib.plan_query(*qargs, 6, cuts=flat)
    roof_ms_mixed, stages_mixed = step_roofline(cfg, sizes, tab, coarse, mixed["stats"], 4, JACOBIAN_EVERY)
    roof_ms_fp64, stages_fp64 = step_roofline(cfg, sizes, tab, coarse, fp64["stats"], 8, JACOBIAN_EVERY)
    flags = [r["stats"]["flags"] for r in (mixed, fp64, gmix, gf64, lagm) if r]
    if schemes:
        flags += [v["flags"] for k, v in schemes.items() if k.startswith("algorithm")]
    if uneven:
        flags += [uneven["mixed"]["flags"], uneven["fp64"]["flags"]]
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
        "graphs": None if gmix is None else {
            "mixed": {"value": rate(gmix["ms_per_step"]), "ms_per_step": gmix["ms_per_step"]},
            "fp64": {"value": rate(gf64["ms_per_step"]), "ms_per_step": gf64["ms_per_step"]},
            "note": "every step's launch sequences replayed as HIP graphs (lp_options.graphs = 1); "
                    "value and ms_per_step above are direct launches"},
        "stages_ms": {"mixed": mixed["stages_ms"], "fp64": fp64["stages_ms"]},
        "refinement": {"scope": "every step of the run (warmup + timed), sticky",
                       "mixed_sweeps_max": mixed["stats"]["ir_sweeps_max"], "mixed_max_sweeps": MAX_IR_MIXED,
                       "mixed_relres_max": mixed["stats"]["ir_relres_max"],
                       "fp64_sweeps_max": fp64["stats"]["ir_sweeps_max"],
                       "fp64_relres_max": fp64["stats"]["ir_relres_max"], "flags": flags,
                       # band factorisations without pivoting: largest growth
                       # factor and smallest pivot relative to the largest entry
                       "lu_monitor": {k: {"growth_local": r["stats"]["lu_growth_local"],
                                          "pivot_local": r["stats"]["lu_pivot_local"],
                                          "growth_coarse": r["stats"]["lu_growth_coarse"],
                                          "pivot_coarse": r["stats"]["lu_pivot_coarse"]}
                                      for k, r in (("mixed", mixed), ("fp64", fp64))},
                       "newton_its_max": [mixed["stats"]["newton_its_max"], fp64["stats"]["newton_its_max"]],
                       "max_newton": MAX_NEWTON, "jacobian_every": JACOBIAN_EVERY},
        "roofline": {"kernel": LU_KERNEL,
                     "bound": bound, "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": gbs / PEAK_HBM_GBS, "traffic": traffic_for(LU_NAME, WORKLOAD),
                     "bytes_per_launch": lu_bytes, "flops_per_launch": lu_flops,
                     "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
                     "mfma_frac": tflops / PEAK_MFMA_FP32_TFLOPS,
                     "avg_launch_ms": lu_ms, "launches": lu_n,
                     "timing": "HIP events around each launch, every stage on one stream (LP_SERIAL=1)",
                     "step": {"mixed": {"roofline_ms": roof_ms_mixed, "measured_ms": mixed["ms_per_step"],
                                        "frac": roof_ms_mixed / mixed["ms_per_step"], "stages": stages_mixed},
                              "fp64": {"roofline_ms": roof_ms_fp64, "measured_ms": fp64["ms_per_step"],
                                       "frac": roof_ms_fp64 / fp64["ms_per_step"], "stages": stages_fp64}}},
    }
    if schemes:
        line["algorithm1_vs_3"] = schemes
    if uneven:
        line["uneven_batch"] = uneven
    if ens:
        line["ensemble"] = ens
    if lagm:
        line["lagged_merged"] = {"ms_per_step": lagm["ms_per_step"], "flags": lagm["stats"]["flags"],
                                 "merge_stage_ms": lagm["stages_ms"].get("merge")}
    if paper:
        line["paper_elements"] = paper
    if not (args.no_cpu or args.lean):
        cores, model = host_cores()
        pool = max(1, min(CPU_POOL_MAX, cores))
        secs1, ref = run_cpu_leg(1)
        secsp, _ = run_cpu_leg(pool) if pool > 1 else (secs1, ref)
        line["cpu_baseline"] = {"value": L * CPU_STEPS / secsp, "unit": "local DoF/s", "cores": pool,
                                "kind": "oracle",
                                "sample": "%d full steps (coarse + local) of the same workload, NumPy/SciPy FP64, "
                                          "local solves over a pool of %d forked processes (one BLAS thread each), "
                                          "%.1f s; host: %d cores available, %s" % (CPU_STEPS, pool, secsp, cores, model),
                                "single_thread_value": L * CPU_STEPS / secs1,
                                "single_thread_seconds": secs1}
        line["accuracy"] = accuracy(cfg, ref)
        if paper:
            line["paper_elements"]["cpu_baseline"] = paper_elements_cpu()
    print(json.dumps(line), flush=True)
    if any(flags):
        print("a refinement, coarse Newton iteration or pivot check failed during the run: flags %s" % flags,
              file=sys.stderr)
        sys.exit(3)


if __name__ == "__main__":
    main()
