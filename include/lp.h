/*
 * lp.h -- C ABI of the MI355X local-parallel finite element library.
 *
 * The library advances the two-grid local parallel scheme for the transient
 * triple-porosity / Navier-Stokes model (Algorithm 3 of Cao, Li, Chen, Du,
 * "A Local Parallel Finite Element Method for Super-Hydrophobic Proppants in a
 * Hydraulic Fracturing System Based on a 2D/3D Transient Triple-Porosity
 * Navier-Stokes Model", Section 5) on one AMD Instinct MI355X (gfx950):
 *
 *   lp_setup        -> domain, nested meshes T_H / T_h, partition {D_j} -> {Omega_j}
 *                      and parameters (Section 2, Section 4 setting, Algorithm 3 Step 2)
 *   lp_coarse_step  -> Algorithm 3 Step 1: one decoupled backward-Euler step on T_H
 *                      (three porous SPD solves + Navier-Stokes by Newton), FP64
 *   lp_local_step   -> Algorithm 3 Steps 3-4: local fine corrections on every
 *                      Omega_j (three porous solves, one Oseen solve) and the
 *                      partition-of-unity correction of the fine solution
 *   lp_get_solution -> copy one field out (merged fine, coarse, or one e_j)
 *
 * Conventions shared by every call
 *   - 2D only in this version (dim = 2).  Porous region (0,1)^2 below the
 *     conduit (0,1)x(1,2); interface Gamma at y = 1 (Example 1, Section 6).
 *   - Each region is an N x N grid of square cells split into the triangles
 *     {(i,j),(i+1,j),(i+1,j+1)} and {(i,j),(i+1,j+1),(i,j+1)}.  P2 nodes are
 *     the half-step lattice (a,b), 0 <= a,b <= 2N, index a + (2N+1) b (the
 *     conduit's vertical index counts up from Gamma); P1 nodes are the
 *     vertices, index i + (N+1) j.
 *   - Vectors crossing the ABI are FP64.  Velocity is component-blocked:
 *     all u_x values, then all u_y values.
 *   - Every device operation is ordered on the HIP stream passed in (a
 *     hipStream_t cast to void*, NULL = default stream).  Only a copy to host
 *     memory synchronises that stream.
 *   - Errors: every call returns an lp_status; on failure lp_last_error()
 *     returns a thread-local message.  No C++ exception crosses the ABI.
 *   - Ownership: input structs and arrays are copied by lp_setup; the caller
 *     may free them afterwards.  The context owns its device memory (taken
 *     from the optional allocator, else hipMalloc) until lp_destroy.
 */
#ifndef LP_H
#define LP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lp_ctx lp_ctx;

typedef enum {
    LP_OK = 0,
    LP_ERR_ARG = 1,          /* invalid argument (sizes, partition, NULL pointer) */
    LP_ERR_STATE = 2,        /* call out of order: setup -> (coarse_step -> local_step)* */
    LP_ERR_ALLOC = 3,        /* device or host allocation failed */
    LP_ERR_DEVICE = 4,       /* a HIP runtime call failed */
    LP_ERR_NOCONV = 5,       /* a solve or refinement did not reach its tolerance;
                                the best iterate is kept and stats.flags is set */
    LP_ERR_UNSUPPORTED = 6   /* valid request this build does not implement */
} lp_status;

/* fields (the paper's u_c, p, p_F, p_f, p_m) */
enum { LP_U = 0, LP_P = 1, LP_PF = 2, LP_PFMI = 3, LP_PM = 4 };
/* levels of lp_get_solution */
enum { LP_MERGED_FINE = 0, LP_COARSE = 1, LP_LOCAL = 2 };
/* arithmetic of the local solves */
enum { LP_FP64 = 0, LP_MIXED = 1 };
/* problems: Example 1's manufactured solution (Section 6); the Example-3-type
 * variant of lp_mini_setup */
enum { LP_MMS_EX1_2D = 0, LP_EX3_2D = 1 };

/* Nested meshes (Section 4: T_h is a uniform refinement of T_H).
 *   n_coarse = 1/H cells per unit length, refine = H/h (integer >= 1). */
typedef struct {
    int32_t dim;             /* 2 */
    int32_t n_coarse;
    int32_t refine;
} lp_mesh;

/* Partition of each region (Algorithm 3 Step 2).
 *   nsub[0], nsub[1]: cores per region along x and y (both regions alike).
 *   overlap: enlargement of each core D_j in fine cells; Omega_j is clipped
 *            to its region and never crosses Gamma.
 *   cuts: NULL for uniform cuts k*N/nsub, else 2*(nsub[0]+1) + 2*(nsub[1]+1)
 *         integers in fine cells, in the order porous-x, porous-y, conduit-x,
 *         conduit-y; each list starts at 0, ends at N and is increasing.
 * Subdomain ids: porous first (x fastest, then y), then conduit. */
typedef struct {
    int32_t nsub[2];
    int32_t overlap;
    const int32_t *cuts;
} lp_partition;

/* Model parameters (Section 2) and the time step.  Index 0,1,2 = F, f, m. */
typedef struct {
    double phi[3], C[3], k[3];
    double mu_tilde, sigma, sigma_star, rho, alpha, eta, nu;
    double dt;
} lp_params;

/* local solver of the per-subdomain systems (Eqs. (5.5)-(5.8)) */
enum { LP_AUTO = 0, LP_DENSE = 1, LP_KRYLOV = 2 };
/* coarse Navier-Stokes step (Algorithm 3 Step 1 (2)) */
enum { LP_NEWTON = 0, LP_SEMI_IMPLICIT = 1 };
/* scheme: the two-grid local parallel method (Algorithm 3) or the one-grid
 * partitioned time stepping it is compared with (Algorithm 1, Section 3.3) */
enum { LP_TWO_GRID = 0, LP_ONE_GRID = 1 };
/* the lagged correction e^n of Eqs. (5.5)-(5.8): the subdomain's own e_j^n,
 * as the equations write it, or the merged correction of Step 4 restricted to
 * the subdomain */
enum { LP_LAG_OWN = 0, LP_LAG_MERGED = 1 };

typedef struct {
    int32_t problem;         /* LP_MMS_EX1_2D (LP_EX3_2D runs through lp_mini_setup only:
                                LP_ERR_UNSUPPORTED here) */
    int32_t precision;       /* LP_FP64 (FP64 factorisation and solves) or
                                LP_MIXED (FP32 factorisation and solves, FP64
                                residuals, iterative refinement) */
    int32_t convection;      /* 1: Navier-Stokes (default); 0: Stokes (drops b_N) */
    int32_t max_ir;          /* refinement sweeps cap (>= 1) */
    double ir_tol;           /* stop when ||b - A x|| <= ir_tol ||b|| per system */
    int32_t max_newton;      /* coarse nonlinear iterations cap per step: chord steps with the
                                exact residual and the inverse of the Jacobian formed at the
                                first iterate of a refresh step; all stop at newton_tol */
    double newton_tol;       /* stop when ||delta|| <= newton_tol ||x|| */
    int32_t jacobian_every;  /* the coarse Jacobian is formed at steps 1, 1 + J, 1 + 2 J, ...
                                and reused in between (0 or 1: every step) */
    int32_t solver;          /* local Oseen solves (Eq. (5.8)): LP_DENSE, the per-step band
                                factorisation (half-bandwidth <= 159); LP_KRYLOV, restarted
                                flexible GMRES(max_iter) in FP64 with the FP64 matrix-free
                                operator, right-preconditioned by restricted additive Schwarz
                                over strips of each box (at most 16 cells wide, 2 cells of
                                overlap) whose Stokes-part band matrices (the operator without
                                b_N) are factored once at setup in the precision of the run;
                                each refinement sweep is one GMRES cycle; LP_AUTO: dense where
                                the half-bandwidth fits, else Krylov.  The porous systems
                                always use the band factorisation. */
    int32_t coarse_ns;       /* LP_NEWTON: the fully implicit coarse step of Algorithm 3
                                Step 1 (2) solved to newton_tol; LP_SEMI_IMPLICIT (convection
                                lagged to u^n, one linear solve): LP_ERR_UNSUPPORTED */
    double krylov_tol;       /* a GMRES cycle stops when its residual estimate is
                                <= krylov_tol ||b|| (the refinement test on the true residual
                                follows) */
    int32_t max_iter;        /* GMRES restart length, 1..64 (the Arnoldi steps of one cycle) */
    int32_t krylov_cycles;   /* GMRES cycles (refinement sweeps) of the Krylov path per local
                                step, 1..max_ir; 0: max_ir */
    int32_t nsamples;        /* parameter samples advanced together (lp_setup's samples[]);
                                0 or 1: one sample.  Several share mesh, partition and dt;
                                every launch then covers all samples' systems, and each
                                sample's fields are what a context of that sample alone
                                computes, bit for bit.  They need the dense local path
                                (LP_DENSE, or LP_AUTO where the band fits) and LP_TWO_GRID
                                (else LP_ERR_UNSUPPORTED); the autotuner then tunes the
                                dense path only */
    int32_t autotune;        /* 1: at the end of lp_setup, time the local Oseen solves on this
                                run's own systems: the band factorisation kernel (three
                                variants) and the band solve prefetch depth are set to the
                                fastest, and under LP_AUTO, where the band path fits, both
                                paths are set up and the faster batch of solves (the dense
                                path's assembly, factorisation and refinement against the
                                Krylov path's GMRES cycles) is kept.  0: fixed defaults. */
    int32_t graphs;          /* 1: every launch sequence that one stream runs between event
                                operations in a step (coarse porous part, coarse Newton
                                chain, prolongation, assembly and factorisation, porous
                                batch, Oseen right-hand sides, Oseen refinement, merge) is
                                captured once per sequence and ring slot (from the third
                                step on) and replayed as a HIP graph on its stream: every
                                argument of a sequence is a function of the slot (the step's
                                time factors are computed on the device), so a replay is the
                                next step of that slot.  Steps with stage timers on
                                (lp_set_timing) use direct launches.  0: direct launches. */
    int32_t scheme;          /* LP_TWO_GRID (default): Algorithm 3.  LP_ONE_GRID: Algorithm 1
                                on the mesh of n_coarse cells (refine must be 1, so T_H = T_h):
                                lp_coarse_step takes its step (the decoupled porous solves
                                and the Navier-Stokes step solved by chord iterations to
                                newton_tol, in FP64), lp_local_step has no work and only
                                completes the step, and LP_MERGED_FINE reads the one grid's
                                fields.  The partition is set up but not used; LP_LOCAL is
                                an LP_ERR_STATE.  The band kernels bound the grid: coarse
                                half-bandwidth 10 n_coarse + 2 <= 175, so n_coarse <= 17. */
    int32_t lagged;          /* LP_LAG_OWN (default): the lagged e^n terms of Eqs. (5.5)-(5.8)
                                (time derivative and exchange) take the subdomain's own
                                correction e_j^n.  LP_LAG_MERGED: after each step's merge
                                (Step 4), every subdomain's porous and velocity corrections
                                are replaced by the merged correction x_h^{n+1} - Pi_h
                                x_H^{n+1} on its lattice (zero on its artificial faces; the
                                conduit pressure correction is not lagged), so the next step
                                starts each subdomain from its neighbours' cores.  The
                                paper's printed Algorithm 3 errors (Table 1, porous columns)
                                are reproduced under this reading with its own elements.
                                No effect with LP_ONE_GRID. */
} lp_options;

/* Optional device allocator (e.g. a framework's caching allocator). */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} lp_allocator;

typedef struct {
    int64_t step;            /* completed local steps */
    int64_t n_porous, n_conduit;      /* subdomains (of one sample) */
    int64_t local_dofs;      /* unknowns solved per local step (all systems of all samples) */
    int64_t max_bw;          /* largest half-bandwidth of a local system */
    int32_t newton_its;      /* Newton iterations of the last coarse step (most over samples) */
    int32_t ir_sweeps;       /* refinement sweeps of the last local step (max over systems) */
    double ir_relres;        /* largest final relative residual of the last local step */
    int32_t flags;           /* sticky over the whole run:
                                bit 0: some local refinement ended above ir_tol;
                                bit 1: some coarse step ended above newton_tol;
                                bit 2: a factorisation met a zero or non-finite pivot, a
                                pivot below one rounding unit of the system's largest
                                entry (|u_kk| <= 2^-23 max|a_ij| in FP32, 2^-52 in FP64)
                                or a growth factor above 2^16 (FP32) / 2^45 (FP64) */
    int32_t newton_its_max;  /* most Newton iterations of any coarse step so far */
    int32_t ir_sweeps_max;   /* most refinement sweeps of any system in any local step so far */
    double ir_relres_max;    /* largest final relative residual of any system in any local step */
    int32_t solver;          /* local Oseen solver in use: LP_DENSE or LP_KRYLOV */
    int32_t tuned;           /* 1 if lp_setup autotuned (lp_options.autotune) */
    int32_t lu_variant;      /* band factorisation kernel of the local Oseen systems */
    int32_t solve_depth;     /* band solve prefetch depth (0: the default per precision) */
    double tune_dense_ms;    /* autotuning: one batch of local Oseen solves by the band path */
    double tune_krylov_ms;   /* ... and by the Krylov path (0 if that path was not set up) */
    int32_t krylov_its;      /* LP_KRYLOV: most GMRES (Arnoldi) steps of any local Oseen
                                system in the last local step, over its cycles */
    int32_t ir_sweeps_porous, ir_sweeps_oseen;   /* ir_sweeps split by system kind */
    double ir_relres_porous, ir_relres_oseen;    /* ir_relres split by system kind */
    /* Band factorisations without pivoting, run-long, over the local systems
     * (Step 3) and the coarse ones (Step 1): the largest growth factor
     * max|u_ij| / max|a_ij| of a system, and the smallest pivot relative to the
     * largest entry of its system, min|u_kk| / max|a_ij| (1 before any). */
    double lu_growth_local, lu_pivot_local;
    double lu_growth_coarse, lu_pivot_coarse;
} lp_stats;

/* Build meshes, partition, reference data and device buffers; interpolate the
 * initial data (t = 0) on both grids and set e_j^0 = I_h x_0 - Pi_h x_H^0 on each
 * Omega_j (zero on artificial faces); factor the constant local porous
 * matrices.  Synchronises `stream` before returning.
 * samples: opt->nsamples parameter sets (one when nsamples is 0 or 1); every
 * sample shares mesh, partition and dt and carries its own Section 2
 * parameters.
 * Errors: LP_ERR_ARG (dim != 2, n_coarse < 1, refine < 1, overlap < 0, bad cuts,
 * non-positive dt or parameters, samples with different dt, unknown option
 * values), LP_ERR_UNSUPPORTED (nsamples > 1 with the Krylov path or
 * LP_ONE_GRID, LP_SEMI_IMPLICIT, a porous, coarse or (LP_DENSE) Oseen
 * half-bandwidth beyond the band kernels' window of 159, or a Krylov strip or
 * system beyond its kernels' limits), LP_ERR_NOCONV (zero or non-finite pivot in
 * the constant porous matrices), LP_ERR_ALLOC, LP_ERR_DEVICE. */
lp_status lp_setup(const lp_mesh *mesh, const lp_partition *part, const lp_params *samples,
                   const lp_options *opt, const lp_allocator *alloc, void *stream,
                   lp_ctx **out);

/* Algorithm 3 Step 1 for t_n -> t_{n+1} on T_H (FP64).  The coarse step runs
 * on an internal stream (it never reads local results); the local Oseen
 * operators of Step 3, which depend only on u_cH^{n+1}, are assembled and
 * factored right after it on a second internal stream, so they overlap the
 * local solves of the previous step.  LP_ERR_STATE if the previous coarse step
 * has not been followed by lp_local_step. */
lp_status lp_coarse_step(lp_ctx *ctx, void *stream);

/* Algorithm 3 Steps 3-4 for t_{n+1}: prolongation, local right-hand sides,
 * local solves, merge, and e_j^n <- e_j^{n+1}.  LP_ERR_STATE unless a coarse
 * step is pending. */
lp_status lp_local_step(lp_ctx *ctx, void *stream);

/* Length (in doubles) of a field at a level.  sub is the subdomain id for
 * LP_LOCAL (its local lattice, Dirichlet nodes included), ignored otherwise. */
lp_status lp_get_size(lp_ctx *ctx, int32_t field, int32_t level, int32_t sub, int64_t *len);

/* Copy a field of one sample into `out` (len doubles; host memory, or device
 * memory when out_is_device != 0).  LP_MERGED_FINE is the corrected fine
 * solution of Algorithm 3 Step 4, x_h = Pi_h x_H + sum_j w_j e_j on each region;
 * LP_COARSE the latest coarse state (Step 1); LP_LOCAL subdomain `sub`'s
 * correction e_j of Step 3 on its local lattice (zero on artificial faces, the
 * lifted boundary values on the physical boundary).  A host copy synchronises
 * `stream`.  Errors: LP_ERR_ARG (sample out of range, unknown field or level,
 * field not carried by that subdomain's region, len too short). */
lp_status lp_get_solution(lp_ctx *ctx, int32_t sample, int32_t field, int32_t level, int32_t sub,
                          double *out, int64_t len, int32_t out_is_device, void *stream);

/* Waits for the device.  Fills `out` and returns LP_OK, or LP_ERR_NOCONV
 * (with `out` filled all the same) when a sticky flag is set: a refinement,
 * a coarse Newton iteration or a pivot check failed in some step so far; the
 * fields hold the best iterates. */
lp_status lp_get_stats(lp_ctx *ctx, lp_stats *out);

/* lp_get_stats restricted to one parameter sample's systems (0 <= sample <
 * nsamples): the coarse Newton iterations of that sample's last step and of
 * its run (newton_its, newton_its_max), flag bit 1 when its last coarse step
 * ended above newton_tol, its last local step's refinement sweeps and final
 * relative residuals (ir_sweeps*, ir_relres*), and local_dofs per sample.
 * Flag bits 0 and 2, the run-long refinement maxima, the factorisation
 * monitor and the solver choice are the context's.  Errors: as lp_get_stats,
 * and LP_ERR_ARG for a sample out of range. */
lp_status lp_get_sample_stats(lp_ctx *ctx, int32_t sample, lp_stats *out);

/* Diagnostic entry for the band kernels of Steps 1 and 3: factor nsys
 * caller-provided band systems without pivoting and solve one right-hand side
 * each, with the library's factorisation (variant as for the local systems:
 * 0 vector units, 8 blocked on MFMA, 9 blocked with lookahead) and band solve.
 * Host arrays, all FP64: band[nsys * n * (2 bw + 1)], system s's entry (i, j)
 * at s n (2 bw + 1) + j (2 bw + 1) + i - j + bw; rhs and x[nsys * n].
 * precision LP_FP64 factors and solves in FP64, LP_MIXED in FP32 (no
 * refinement: x is the plain FP32 solve).  Outputs: *flags (bit 2 as in
 * lp_stats), *growth and *pivot_min over the systems (as the lu_* fields of
 * lp_stats).  Allocates and frees device memory; synchronous.
 * Errors: LP_ERR_ARG (sizes, precision, variant), LP_ERR_UNSUPPORTED (bw beyond
 * the kernels' window of 175 for variant 0, 160 for 8 and 9), LP_ERR_DEVICE. */
lp_status lp_band_factor_solve(int32_t nsys, int32_t n, int32_t bw, const double *band, const double *rhs,
                               double *x, int32_t precision, int32_t variant, int32_t *flags,
                               double *growth, double *pivot_min);

/* Host-only partition queries (no device needed), for bit-exact index parity.
 *   which = 0: subdomain table, 9 int64 per subdomain:
 *              region, x0, x1, y0, y1 (Omega box), dx0, dx1, dy0, dy1 (core D)
 *   which = 1: P2 node class of subdomain `sub`, local lattice order:
 *              0 free, 1 physical Dirichlet, 2 artificial (zero)
 *   which = 2: P1 vertex class of subdomain `sub` (0 free, 2 artificial)
 *   which = 3: band-system unknown of each local P2 node of `sub`
 *              (porous: scalar index; conduit: index of u_x, u_y follows), -1 if fixed
 *   which = 4: band-system unknown of each local P1 vertex of conduit `sub`, -1 if fixed
 *   which = 5: per subdomain: number of unknowns and half-bandwidth (2 int64 each)
 *   which = 6: the coarse systems on T_H: unknowns and half-bandwidth of one
 *              porous pressure system, then of the Navier-Stokes system
 *   which = 7: the strips of the Krylov path's preconditioner for a strip
 *              width of `sub` cells, 7 int64 per strip: parent conduit
 *              system (0-based among the conduit subdomains), x0, x1, y0, y1,
 *              unknowns, half-bandwidth
 * For which = 1..4, sub = -1 returns the tables of every subdomain (of every
 * conduit subdomain for which = 4) concatenated in id order. 
 * `needed` receives the required length; nothing is written if len is short. */
lp_status lp_plan_query(const lp_mesh *mesh, const lp_partition *part, int32_t which,
                        int32_t sub, int64_t *out, int64_t len, int64_t *needed);

/* The same tables as lp_plan_query, read from a context's own plan (the
 * numbering its kernels use).  `needed` receives the required length; nothing
 * is written if len is short.  Errors: LP_ERR_ARG. */
lp_status lp_get_index_map(lp_ctx *ctx, int32_t which, int32_t sub, int64_t *out, int64_t len,
                           int64_t *needed);

/* Stage timers: HIP events recorded around the launches of the stages
 * selected in `mask`, on the stream each stage runs on (bit i = stage i below;
 * the coarse step, the prolongation, the porous batch and the Oseen assembly
 * and factorisation run on the context's internal streams, the rest on the
 * caller's); 0 turns
 * them off.  Setting a mask clears the accumulators.  lp_get_timing waits for
 * the recorded events and returns, per stage, the summed milliseconds and the
 * number of timed launches (arrays of length n <= LP_T_COUNT). */
enum {
    LP_T_PROLONG = 0,        /* coarse -> fine prolongation for the Oseen assembly, the local
                                Oseen stage and the merge (internal stream, before the assembly) */
    LP_T_POR_RHS = 1,        /* local porous right-hand sides */
    LP_T_POR_SOLVE = 2,      /* local porous band solves (all refinement sweeps) */
    LP_T_POR_RES = 3,        /* local porous FP64 residuals */
    LP_T_OSE_RHS = 4,        /* local Oseen right-hand sides */
    LP_T_OSE_ASM = 5,        /* local Oseen band assembly (incl. prolonging u_cH and clearing the band) */
    LP_T_OSE_LU = 6,         /* local Oseen band factorisation (one kernel launch) */
    LP_T_OSE_SOLVE = 7,      /* local Oseen band solves (all sweeps) */
    LP_T_OSE_RES = 8,        /* local Oseen FP64 residuals */
    LP_T_MERGE = 9,          /* finalize + partition-of-unity merge */
    LP_T_COARSE = 10,        /* the whole coarse step */
    LP_T_WAIT_COARSE = 11,   /* local step start waiting for its coarse step */
    LP_T_WAIT_FAC = 12,      /* local Oseen solves waiting for their factors */
    LP_T_WAIT_POR = 13,      /* merge waiting for the porous batch */
    LP_T_COUNT = 14
};
lp_status lp_set_timing(lp_ctx *ctx, uint32_t mask);
lp_status lp_get_timing(lp_ctx *ctx, double *ms, int64_t *launches, int32_t n);

/* lp_local_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with the refinement scratch (residual-norm
 * partials and last-block tickets of the porous and Oseen batches) in a
 * file-scope device array of LP_NOALLOC_SCRATCH_BYTES (8 MiB) that each
 * device holds until the process ends, instead of context buffers.  Calls no
 * allocator; its tickets are cleared by a small kernel on each call.  Every
 * call on one device shares that array: calls of different contexts that
 * overlap on one device race.  Errors: as lp_local_step, and
 * LP_ERR_UNSUPPORTED when the problem's scratch (all samples' systems)
 * exceeds the array. */
lp_status lp_local_step_noalloc(lp_ctx *ctx, void *stream);

/* Checkpoint and resume of a run between steps (no coarse step pending).
 * The state is what the next steps read: the coarse states of the last
 * levels (Algorithm 3 Step 1 lags them and starts Newton from them), the
 * local corrections e_j^n that Step 3 reads back (Eqs. (5.5)-(5.8)), the
 * merged fields of Step 4, the coarse Jacobian inverse in use when
 * jacobian_every > 1, the time-level counters, the coarse Newton status and
 * the sticky flags and run-long maxima of lp_get_stats; prolongations,
 * factorisations and right-hand sides are rebuilt by the next step.  A
 * context set up with the same mesh, partition, samples (parameters and dt)
 * and options continues from it exactly where the saving one would have:
 * the same fields, bit for bit, when the same kernel variants run (the
 * autotuner may choose others on another run).
 *   lp_state_size: bytes of the state of `ctx` (no device call).
 *   lp_save_state: writes it into `buf` (host memory, `len` bytes, owned by
 *     the caller); waits for `stream` and the device.
 *   lp_load_state: replaces the state of `ctx` by `buf`'s; the step count
 *     continues from the saved one.
 * Errors: LP_ERR_ARG (NULL, `len` too short, a buffer that is not a saved
 * state or was saved by a context of another mesh, partition, sample set,
 * precision, scheme or jacobian_every), LP_ERR_STATE (a coarse step is
 * pending), LP_ERR_DEVICE. */
lp_status lp_state_size(lp_ctx *ctx, int64_t *bytes);
lp_status lp_save_state(lp_ctx *ctx, void *buf, int64_t len, void *stream);
lp_status lp_load_state(lp_ctx *ctx, const void *buf, int64_t len, void *stream);

void lp_destroy(lp_ctx *ctx);

/* The paper's own discretisation on the device (Section 6, first paragraph:
 * MINI elements, P1b-P1, in the conduit and P1 elements for the porous
 * pressures) with Algorithm 1 (partitioned time stepping, Section 3.3) on one
 * grid of n cells per unit length, for Example 1's manufactured solution
 * (Section 6), FP64 throughout.  Per step t_n -> t_{n+1} = (n+1) dt:
 *   1. the three porous P1 systems with the lagged exchange terms and the
 *      lagged Gamma flux u^n . n_c (their matrices are constant: factored
 *      once at setup);
 *   2. backward-Euler Navier-Stokes on the MINI space with the lagged p_F^n
 *      on Gamma, from (u^n, p^n) with the boundary values of t_{n+1}, by chord
 *      iterations (the Jacobian of the step's first iterate, applied to the
 *      exact residual of every iterate) to a relative update <= 1e-13 (at
 *      most 30 iterations).
 * The same model, coefficients and time levels as lp_setup's (sources and
 * Dirichlet data at t_{n+1}); initial data: vertex values of the exact
 * fields, and each element's bubble coefficient chosen so that the
 * element's value at its centroid is exact.  The bubble is 27 l0 l1 l2
 * (value 1 at the centroid); elements are numbered 2 (i + n j) + t in cell
 * (i, j), t = 0 the triangle (0,0),(1,0),(1,1) of the cell, t = 1 the
 * triangle (0,0),(1,1),(0,1).
 * Fields read back by lp_mini_get (host arrays owned by the caller):
 *   LP_PF, LP_PFMI, LP_PM: (n+1)^2 porous vertex values, index i + (n+1) j;
 *   LP_P: (n+1)^2 conduit vertex values (j counted up from Gamma);
 *   LP_U: u_x then u_y, each (n+1)^2 vertex values then one bubble
 *         coefficient per element: 2 ((n+1)^2 + 2 n^2) values.
 * problem LP_EX3_2D is an Example-3-type variant (Section 6, Example 3) on
 * the same two squares: the porous region's outer boundary is Gamma_in with
 * fixed p_F = 1.0e3, p_f = 1.6e3, p_m = 4.0e3 (also the initial porous state);
 * there are no sources; the conduit is Stokes (no convection) and starts at
 * rest; its side walls x = 0, 1 are cased (u = 0, end points included); the
 * rest of its top y = 2 is the outflow boundary (T(u, p) n = 0, natural).
 * Fluid enters the conduit only through Gamma.  Boundary data are constant
 * in time.
 * lp_mini_setup: `problem` is LP_MMS_EX1_2D or LP_EX3_2D; `device` is a HIP
 *   device id; samples[nsamples] (host, read during the call) hold the
 *   parameters and dt of independent runs advanced together (a parameter
 *   sweep: every launch covers all samples' systems, and each sample's fields
 *   are bit for bit those of a one-sample context with its parameters); the
 *   samples share dt.  Errors: LP_ERR_ARG (NULL, nsamples < 1, dt <= 0 or
 *   differing, k_F, mu_tilde or rho <= 0, n < 2: with n = 1 every conduit
 *   vertex has Dirichlet velocity and the pressure keeps a free constant),
 *   LP_ERR_DEVICE,
 *   LP_ERR_UNSUPPORTED (the Navier-Stokes half-bandwidth, 7 n + 16 for n >= 2,
 *   beyond the band kernels' window of 175: n <= 22), LP_ERR_ALLOC.
 * lp_mini_step: advances nsteps steps, synchronously.  LP_ERR_NOCONV when a
 *   Newton solve reached its cap (flags bit 1) or a factorisation met a
 *   pivot below the rounding of its matrix (bit 2); the flags are sticky and
 *   the state advances all the same.
 * lp_mini_get: copies `field` of `sample` into out[len]; *needed (if not
 *   NULL) receives its length; out = NULL only queries it.  LP_ERR_ARG for a
 *   sample out of range, an unknown field or a short buffer.
 * lp_mini_stats: steps taken, the most iterations of any step (any sample),
 *   flags, and the
 *   summed HIP-event time (ms) and count of the Navier-Stokes factorisations
 *   (any output may be NULL). */
typedef struct lp_mini lp_mini;
lp_status lp_mini_setup(int32_t n, int32_t problem, const lp_params *samples, int32_t nsamples, int32_t device,
                        lp_mini **out);
lp_status lp_mini_step(lp_mini *ctx, int32_t nsteps);
lp_status lp_mini_get(lp_mini *ctx, int32_t sample, int32_t field, double *out, int64_t len, int64_t *needed);
lp_status lp_mini_stats(lp_mini *ctx, int32_t *steps, int32_t *newton_its_max, int32_t *flags, double *lu_ms,
                        int64_t *lu_launches);
void lp_mini_destroy(lp_mini *ctx);

const char *lp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LP_H */
