"""ctypes binding of liblp.so (argument marshalling only: every step of the
scheme runs in the library's HIP kernels).

PyTorch supplies the HIP stream and, optionally, device memory through its
caching allocator.  Importing this module loads the library and raises if it
has not been built; there is no fallback implementation.
"""
import ctypes
import os
from ctypes import (CFUNCTYPE, POINTER, Structure, byref, c_char_p, c_double, c_int32, c_int64,
                    c_size_t, c_void_p)

import numpy as np
# torch first: its bundled HIP runtime (same soname as the system one) must be
# the one liblp.so binds to, so the library and torch share devices and streams
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblp.so")

LP_U, LP_P, LP_PF, LP_PFMI, LP_PM = range(5)
LP_MERGED_FINE, LP_COARSE, LP_LOCAL = range(3)
LP_FP64, LP_MIXED = 0, 1
FIELD = {"u": LP_U, "p": LP_P, "pF": LP_PF, "pf": LP_PFMI, "pm": LP_PM}
LEVEL = {"merged": LP_MERGED_FINE, "coarse": LP_COARSE, "local": LP_LOCAL}
STATUS = {0: "LP_OK", 1: "LP_ERR_ARG", 2: "LP_ERR_STATE", 3: "LP_ERR_ALLOC", 4: "LP_ERR_DEVICE",
          5: "LP_ERR_NOCONV", 6: "LP_ERR_UNSUPPORTED"}

LP_AUTO, LP_DENSE, LP_KRYLOV = range(3)
LP_NEWTON, LP_SEMI_IMPLICIT = range(2)
SOLVER = {"auto": LP_AUTO, "dense": LP_DENSE, "krylov": LP_KRYLOV}
COARSE_NS = {"newton": LP_NEWTON, "semi_implicit": LP_SEMI_IMPLICIT}
LP_TWO_GRID, LP_ONE_GRID = range(2)
SCHEME = {"two_grid": LP_TWO_GRID, "one_grid": LP_ONE_GRID}
LAGGED = {"own": 0, "merged": 1}
LP_ERR_NOCONV = 5

EXPORTS = ["lp_setup", "lp_coarse_step", "lp_local_step", "lp_get_size", "lp_get_solution",
           "lp_get_stats", "lp_get_sample_stats", "lp_plan_query", "lp_get_index_map", "lp_set_timing", "lp_get_timing",
           "lp_local_step_noalloc", "lp_band_factor_solve", "lp_state_size", "lp_save_state",
           "lp_load_state", "lp_mini_setup", "lp_mini_step", "lp_mini_get", "lp_mini_stats", "lp_mini_destroy",
           "lp_destroy", "lp_last_error"]
# stage timer indices (LP_T_* in lp.h)
STAGES = ["prolong", "por_rhs", "por_solve", "por_res", "ose_rhs", "ose_asm", "ose_lu", "ose_solve",
          "ose_res", "merge", "coarse", "wait_coarse", "wait_fac", "wait_por"]


class LpMesh(Structure):
    _fields_ = [("dim", c_int32), ("n_coarse", c_int32), ("refine", c_int32)]


class LpPartition(Structure):
    _fields_ = [("nsub", c_int32 * 2), ("overlap", c_int32), ("cuts", POINTER(c_int32))]


class LpParams(Structure):
    _fields_ = [("phi", c_double * 3), ("C", c_double * 3), ("k", c_double * 3),
                ("mu_tilde", c_double), ("sigma", c_double), ("sigma_star", c_double),
                ("rho", c_double), ("alpha", c_double), ("eta", c_double), ("nu", c_double),
                ("dt", c_double)]


class LpOptions(Structure):
    _fields_ = [("problem", c_int32), ("precision", c_int32), ("convection", c_int32),
                ("max_ir", c_int32), ("ir_tol", c_double), ("max_newton", c_int32),
                ("newton_tol", c_double), ("jacobian_every", c_int32), ("solver", c_int32),
                ("coarse_ns", c_int32), ("krylov_tol", c_double), ("max_iter", c_int32),
                ("krylov_cycles", c_int32), ("nsamples", c_int32), ("autotune", c_int32), ("graphs", c_int32),
                ("scheme", c_int32), ("lagged", c_int32)]


ALLOC_FN = CFUNCTYPE(c_void_p, c_size_t, c_void_p)
FREE_FN = CFUNCTYPE(None, c_void_p, c_void_p)


class LpAllocator(Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", c_void_p)]


class LpStats(Structure):
    _fields_ = [("step", c_int64), ("n_porous", c_int64), ("n_conduit", c_int64),
                ("local_dofs", c_int64), ("max_bw", c_int64), ("newton_its", c_int32),
                ("ir_sweeps", c_int32), ("ir_relres", c_double), ("flags", c_int32),
                ("newton_its_max", c_int32), ("ir_sweeps_max", c_int32), ("ir_relres_max", c_double),
                ("solver", c_int32), ("tuned", c_int32), ("lu_variant", c_int32), ("solve_depth", c_int32),
                ("tune_dense_ms", c_double), ("tune_krylov_ms", c_double), ("krylov_its", c_int32),
                ("ir_sweeps_porous", c_int32), ("ir_sweeps_oseen", c_int32), ("ir_relres_porous", c_double),
                ("ir_relres_oseen", c_double), ("lu_growth_local", c_double), ("lu_pivot_local", c_double),
                ("lu_growth_coarse", c_double), ("lu_pivot_coarse", c_double)]


class LpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("liblp.so is not built (%s); run python -m paper_2311_05170_amd.build" % path)
    lib = ctypes.CDLL(path)
    lib.lp_setup.argtypes = [POINTER(LpMesh), POINTER(LpPartition), POINTER(LpParams), POINTER(LpOptions),
                             POINTER(LpAllocator), c_void_p, POINTER(c_void_p)]
    lib.lp_coarse_step.argtypes = [c_void_p, c_void_p]
    lib.lp_local_step.argtypes = [c_void_p, c_void_p]
    lib.lp_local_step_noalloc.argtypes = [c_void_p, c_void_p]
    lib.lp_get_size.argtypes = [c_void_p, c_int32, c_int32, c_int32, POINTER(c_int64)]
    lib.lp_get_solution.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_int32, POINTER(c_double),
                                    c_int64, c_int32, c_void_p]
    lib.lp_get_stats.argtypes = [c_void_p, POINTER(LpStats)]
    lib.lp_get_sample_stats.argtypes = [c_void_p, c_int32, POINTER(LpStats)]
    lib.lp_plan_query.argtypes = [POINTER(LpMesh), POINTER(LpPartition), c_int32, c_int32,
                                  POINTER(c_int64), c_int64, POINTER(c_int64)]
    lib.lp_get_index_map.argtypes = [c_void_p, c_int32, c_int32, POINTER(c_int64), c_int64, POINTER(c_int64)]
    lib.lp_set_timing.argtypes = [c_void_p, ctypes.c_uint32]
    lib.lp_get_timing.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int64), c_int32]
    lib.lp_band_factor_solve.argtypes = [c_int32, c_int32, c_int32, POINTER(c_double), POINTER(c_double),
                                         POINTER(c_double), c_int32, c_int32, POINTER(c_int32), POINTER(c_double),
                                         POINTER(c_double)]
    lib.lp_state_size.argtypes = [c_void_p, POINTER(c_int64)]
    lib.lp_save_state.argtypes = [c_void_p, c_void_p, c_int64, c_void_p]
    lib.lp_load_state.argtypes = [c_void_p, c_void_p, c_int64, c_void_p]
    lib.lp_destroy.argtypes = [c_void_p]
    lib.lp_destroy.restype = None
    lib.lp_last_error.restype = c_char_p
    lib.lp_mini_setup.argtypes = [c_int32, c_int32, POINTER(LpParams), c_int32, c_int32, POINTER(c_void_p)]
    lib.lp_mini_step.argtypes = [c_void_p, c_int32]
    lib.lp_mini_get.argtypes = [c_void_p, c_int32, c_int32, POINTER(c_double), c_int64, POINTER(c_int64)]
    lib.lp_mini_stats.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32), POINTER(c_double),
                                  POINTER(c_int64)]
    lib.lp_mini_destroy.argtypes = [c_void_p]
    for name in EXPORTS[:-2]:
        getattr(lib, name).restype = c_int32
    lib.lp_mini_destroy.restype = None
    return lib


_LIB = load()


def _check(status):
    if status != 0:
        raise LpError(status, _LIB.lp_last_error().decode())


def _structs(n_coarse, refine, nsub, overlap, cuts):
    mesh = LpMesh(2, int(n_coarse), int(refine))
    part = LpPartition()
    part.nsub[0], part.nsub[1] = int(nsub[0]), int(nsub[1])
    part.overlap = int(overlap)
    keep = None
    if cuts is not None:
        keep = (c_int32 * len(cuts))(*[int(v) for v in cuts])
        part.cuts = ctypes.cast(keep, POINTER(c_int32))
    return mesh, part, keep


def band_factor_solve(band, rhs, precision="fp64", variant=9):
    """Factor and solve caller-provided band systems with the library's band
    kernels (lp_band_factor_solve).  band: (nsys, n, 2 bw + 1) FP64, entry
    (i, j) of system s at band[s, j, i - j + bw]; rhs: (nsys, n).  Returns
    (x, flags, growth, pivot_min)."""
    band = np.ascontiguousarray(band, dtype=np.float64)
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    nsys, n, ld = band.shape
    x = np.zeros((nsys, n))
    flags, growth, pivot = c_int32(0), c_double(0.0), c_double(0.0)
    dp = lambda a: a.ctypes.data_as(POINTER(c_double))  # noqa: E731
    _check(_LIB.lp_band_factor_solve(nsys, n, (ld - 1) // 2, dp(band), dp(rhs), dp(x), LP_MIXED if precision == "mixed" else LP_FP64,
                                     int(variant), byref(flags), byref(growth), byref(pivot)))
    return x, flags.value, growth.value, pivot.value


def plan_query(n_coarse, refine, nsub, overlap, which, sub=0, cuts=None):
    """Host-only partition tables (no device needed); see lp_plan_query."""
    mesh, part, keep = _structs(n_coarse, refine, nsub, overlap, cuts)
    need = c_int64(0)
    _check(_LIB.lp_plan_query(byref(mesh), byref(part), which, sub, None, 0, byref(need)))
    out = np.zeros(max(need.value, 1), dtype=np.int64)
    _check(_LIB.lp_plan_query(byref(mesh), byref(part), which, sub,
                              out.ctypes.data_as(POINTER(c_int64)), need.value, byref(need)))
    return out[:need.value]


def _params(prm, dt):
    p = LpParams()
    for i in range(3):
        p.phi[i], p.C[i], p.k[i] = prm["phi"][i], prm["C"][i], prm["k"][i]
    for key in ("mu_tilde", "sigma", "sigma_star", "rho", "alpha", "eta", "nu"):
        setattr(p, key, float(prm[key]))
    p.dt = float(dt)
    return p


class LocalParallel:
    """One run of the local parallel scheme on the current HIP device.

    precision: "mixed" (FP32 factorisations, FP64 refinement) or "fp64".
    """

    def __init__(self, n_coarse, refine, nsub, overlap, prm, dt, cuts=None, precision="mixed",
                 convection=True, max_ir=8, ir_tol=None, max_newton=16, newton_tol=1e-13,
                 jacobian_every=1, solver="auto", coarse_ns="newton", samples=None,
                 krylov_restart=30, krylov_tol=None, krylov_cycles=0, autotune=False, graphs=False,
                 scheme="two_grid", torch_allocator=True, lagged="own"):
        import torch
        self._torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible")
        mesh, part, keep = _structs(n_coarse, refine, nsub, overlap, cuts)
        opt = LpOptions()
        opt.problem = 0
        opt.precision = LP_MIXED if precision == "mixed" else LP_FP64
        opt.convection = 1 if convection else 0
        opt.max_ir = int(max_ir)
        opt.ir_tol = float(ir_tol if ir_tol is not None else (1e-10 if precision == "mixed" else 1e-12))
        opt.max_newton = int(max_newton)
        opt.newton_tol = float(newton_tol)
        opt.jacobian_every = int(jacobian_every)
        opt.solver = SOLVER[solver]
        opt.coarse_ns = COARSE_NS[coarse_ns]
        # a GMRES cycle stops a decade below the refinement tolerance, so the
        # true residual test that follows it passes after one cycle
        opt.krylov_tol = float(krylov_tol if krylov_tol is not None else 0.1 * opt.ir_tol)
        opt.max_iter = int(krylov_restart)
        opt.krylov_cycles = int(krylov_cycles)
        opt.autotune = 1 if autotune else 0
        opt.graphs = 1 if graphs else 0
        opt.scheme = SCHEME[scheme]
        opt.lagged = LAGGED[lagged] if lagged in LAGGED else int(lagged)
        plist = [prm] if samples is None else list(samples)
        opt.nsamples = len(plist)
        params = (LpParams * len(plist))(*[_params(q, dt) for q in plist])
        self._alloc = None
        alloc_ptr = None
        if torch_allocator:
            def _a(nbytes, user):
                return torch.cuda.caching_allocator_alloc(int(nbytes))

            def _f(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)
            self._cb = (ALLOC_FN(_a), FREE_FN(_f))
            self._alloc = LpAllocator(self._cb[0], self._cb[1], None)
            alloc_ptr = byref(self._alloc)
        self.stream = torch.cuda.current_stream()
        handle = c_void_p()
        _check(_LIB.lp_setup(byref(mesh), byref(part), params, byref(opt),
                             alloc_ptr, c_void_p(self.stream.cuda_stream), byref(handle)))
        self._h = handle
        self.n_sub = 2 * nsub[0] * nsub[1]

    def _s(self):
        return c_void_p(self.stream.cuda_stream)

    def coarse_step(self):
        _check(_LIB.lp_coarse_step(self._h, self._s()))

    def local_step(self):
        _check(_LIB.lp_local_step(self._h, self._s()))

    def step(self):
        self.coarse_step()
        self.local_step()

    def size(self, field, level="merged", sub=0):
        n = c_int64(0)
        _check(_LIB.lp_get_size(self._h, FIELD[field], LEVEL[level], sub, byref(n)))
        return n.value

    def solution(self, field, level="merged", sub=0, sample=0):
        n = self.size(field, level, sub)
        out = np.zeros(n, dtype=np.float64)
        _check(_LIB.lp_get_solution(self._h, sample, FIELD[field], LEVEL[level], sub,
                                    out.ctypes.data_as(POINTER(c_double)), n, 0, self._s()))
        return out

    def solution_device(self, field, level="merged", sub=0, sample=0):
        torch = self._torch
        n = self.size(field, level, sub)
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(_LIB.lp_get_solution(self._h, sample, FIELD[field], LEVEL[level], sub,
                                    ctypes.cast(out.data_ptr(), POINTER(c_double)), n, 1, self._s()))
        return out

    def save_state(self):
        """The run's state between steps (lp_save_state) as bytes."""
        n = c_int64(0)
        _check(_LIB.lp_state_size(self._h, byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(_LIB.lp_save_state(self._h, buf, n.value, self._s()))
        return buf.raw

    def load_state(self, state):
        """Continue from a state saved by a context built with the same
        arguments (lp_load_state)."""
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        _check(_LIB.lp_load_state(self._h, buf, len(state), self._s()))

    def index_map(self, which, sub=0):
        """The context's own partition and numbering tables (see lp_plan_query)."""
        need = c_int64(0)
        _check(_LIB.lp_get_index_map(self._h, which, sub, None, 0, byref(need)))
        out = np.zeros(max(need.value, 1), dtype=np.int64)
        _check(_LIB.lp_get_index_map(self._h, which, sub, out.ctypes.data_as(POINTER(c_int64)),
                                     need.value, byref(need)))
        return out[:need.value]

    def stats(self, sample=None):
        """Run statistics; flags are sticky.  A set flag (lp_get_stats returns
        LP_ERR_NOCONV) is reported in the dict, not raised.  With a sample
        index, that sample's Newton and refinement statistics
        (lp_get_sample_stats)."""
        s = LpStats()
        if sample is None:
            st = _LIB.lp_get_stats(self._h, byref(s))
        else:
            st = _LIB.lp_get_sample_stats(self._h, int(sample), byref(s))
        if st not in (0, LP_ERR_NOCONV):
            _check(st)
        return {k: getattr(s, k) for k, _ in LpStats._fields_}

    def set_timing(self, stages):
        """Turn the stage timers on for the named stages (empty = off); clears them."""
        mask = 0
        for name in stages:
            mask |= 1 << STAGES.index(name)
        _check(_LIB.lp_set_timing(self._h, mask))

    def timing(self):
        """{stage: (summed ms, timed launches)} since the last set_timing."""
        ms = (c_double * len(STAGES))()
        cnt = (c_int64 * len(STAGES))()
        _check(_LIB.lp_get_timing(self._h, ms, cnt, len(STAGES)))
        return {STAGES[i]: (ms[i], int(cnt[i])) for i in range(len(STAGES))}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _LIB.lp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MiniAlgorithm1:
    """Algorithm 1 with the paper's MINI + P1 elements on one grid of n cells
    per unit length, on the device (lp_mini_*).  Fields come back in the
    layouts lp.h states (vertex values, then one bubble per element for u)."""

    def __init__(self, n, prm, dt, device=0, problem="ex1", samples=None):
        self._h = c_void_p()
        plist = samples if samples else [prm]
        params = (LpParams * len(plist))(*[_params(q, dt) for q in plist])
        _check(_LIB.lp_mini_setup(int(n), {"ex1": 0, "ex3": 1}[problem], params, len(plist), int(device),
                                  byref(self._h)))
        self.nsamples = len(plist)
        self.n = int(n)

    def step(self, nsteps=1):
        _check(_LIB.lp_mini_step(self._h, int(nsteps)))

    def solution(self, field, sample=0):
        need = c_int64(0)
        _check(_LIB.lp_mini_get(self._h, int(sample), FIELD[field], None, 0, byref(need)))
        out = np.zeros(need.value, dtype=np.float64)
        _check(_LIB.lp_mini_get(self._h, int(sample), FIELD[field], out.ctypes.data_as(POINTER(c_double)),
                                need.value, None))
        return out

    def stats(self):
        st, its, fl, lms, lun = c_int32(0), c_int32(0), c_int32(0), c_double(0.0), c_int64(0)
        _check(_LIB.lp_mini_stats(self._h, byref(st), byref(its), byref(fl), byref(lms), byref(lun)))
        return dict(step=st.value, newton_its_max=its.value, flags=fl.value, lu_ms=lms.value, lu_launches=lun.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _LIB.lp_mini_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
