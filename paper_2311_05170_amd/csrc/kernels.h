// Kernel argument blocks and launch wrappers (see kernels.hip).
#pragma once

#include "lp_internal.h"

namespace lp {

struct ProlongArgs {
    const double *src[6];         // sample 0's fields in the per-sample arena
    double *dst[6];
    int nfields;
    int NH, Nh, k;
    long long zs = 0;             // arena stride between samples (doubles); grid row = sample
};

// Start of a refinement, written by the local right-hand side kernels beside
// b: x = 0 and r = b on every row, and the per-system flags cleared (null:
// not written)
struct IrStart {
    double *x, *r;
    int *conv;
    double *relres;
    int *sweeps;
};

struct PorousArgs {
    const SysDesc *sys;
    const int8_t *cls2;
    const int32_t *dof2;
    const double *P1[3];          // background at t_{n+1} on the grid lattice (NULL = 0)
    const double *P0[3];          // background at t_n (NULL = 0)
    const double *ex[3];          // spatial parts of the exact p_F, p_f, p_m
    const double *load[3][2];     // source loads (cos t, sin t parts)
    const double *Uy0;            // conduit u_y at t_n on the same grid (Gamma flux), NULL = none
    const double *e_old;          // previous corrections (local lattices)
    double *e_new;
    double *b;
    const double *tf;             // device: cos t_{n+1}, sin t_{n+1}, cos^2 t_{n+1}
    IrStart ir;                   // three flags per system
    const Coef *co = nullptr;     // the context's coefficients (device)
};

struct ResidualArgs {
    const SysDesc *sys;
    const int32_t *dof2;
    const double *x;
    const double *b;
    double *r;
    int *conv;
    double *relres;
    int *sweeps;
    double tol;
    const int *skip;
    double *part;                 // per-(system, tile) partial norms: 2 * tstride doubles per id
    int *ticket;                  // per-box arrival counters (at the box's first id), zero between launches
    const Coef *co = nullptr;     // the context's coefficients (device)
    int tstride = 0;              // tiles per id in part (at least any box's tile count)
};

// Refinement outcome of a batch, folded into run-long totals by the finalize
// kernels (null acc: not recorded): per system id its convergence flag, sweep
// count and final relative residual; a system that ended unconverged sets bit
// 0 of *flags, the largest sweep count and residual of the run so far are kept
// (the residual as the bit pattern of a non-negative double, whose integer
// order is its numeric order).
struct IrTotals {
    const int *conv;
    const int *sweeps;
    const double *relres;
    int ids_per_sys;
    int *flags;
    int *max_sweeps;
    unsigned long long *max_relres;
};

struct FinalizeArgs {
    const SysDesc *sys;
    const int32_t *dof2;
    const int32_t *dof1;
    const double *x;
    double *e_new;
    double *e_new1;
    const int *skip;
    IrTotals acc;
};

template <typename T>
struct AssembleArgs {
    const SysDesc *sys;
    const int32_t *dof2;
    T *band;
    const Coef *co = nullptr;     // the context's coefficients (device)
};

struct OseenArgs {
    const SysDesc *sys;
    const int8_t *cls2;
    const int32_t *dof2;
    const int8_t *cls1;
    const int32_t *dof1;
    const double *W1[2];          // velocity background at t_{n+1} (Newton iterate on T_H)
    const double *W0[2];          // velocity background at t_n (NULL = 0)
    const double *Pp;             // pressure background at t_{n+1} (P1 lattice)
    const double *ex[2];          // spatial parts of the exact u
    const double *load[2][3];     // source loads (cos, sin, cos^2 parts)
    const double *PF0;            // porous p_F at t_n (Gamma terms)
    const double *e_old;          // previous velocity corrections (NULL = 0)
    double *e_new;
    double *e_new1;
    double *b;
    const double *tf;             // device: cos t_{n+1}, sin t_{n+1}, cos^2 t_{n+1}
    const int *skip;
    IrStart ir;                   // one flag per system
    const Coef *co = nullptr;     // the context's coefficients (device)
};

template <typename T>
struct OseenApplyArgs {
    const SysDesc *sys;
    const int8_t *cls2;
    const int32_t *dof2;
    const int32_t *dof1;
    const double *W1[2];
    const double *x;
    const double *b;
    double *r;
    T *band;
    int *conv;
    double *relres;
    int *sweeps;
    double tol;
    const int *skip;
    double *part;                 // residual mode: partial norms and counters as in ResidualArgs
    int *ticket;
    int tstride = 0;              // residual mode: tiles per system in part
    int no_convection;            // assembly: leave out b_N (the Stokes part of the operator)
    const Coef *co = nullptr;     // the context's coefficients (device)
    int first_write = 0;          // assembly: the band was cleared once and its pattern is fixed (see k_oseen_assemble)
};

struct BandSys {
    long long off;                // band offset of the first matrix
    long long stride;             // distance between the matrices of one system
    long long vec;                // vector offset of the first right-hand side
    long long foff;               // factor offset of the first matrix
    long long fstride;            // distance between the factors of the matrices of one system
    int n, bw, nrhs;
    int ldf;                      // factor column length, 64 x (solve registers per lane)
};

// window registers per lane of the band solve for a half-bandwidth (0: unsupported)
// Factor layout shared by the factorisations and the solves.  The solve keeps
// a window of R = 64 NR rows in NR registers per lane, in halves of 32 rows:
// row i sits in slot s = i mod R, half h = s / 32 (register h / 2, lanes
// 32 (h mod 2) + (s mod 32)).  A factor column holds ldf = R values, lane l's
// NR values contiguous: slot s at fac_pos(s) = lane(s) NR + register(s).
//   Lr[k ldf + fac_pos(i mod R)] = L(i, k),                 k < i <= k + bw
//   Ur[(n-1-j) ldf + fac_pos((n-1-i) mod R)] = U(i, j) / U(i, i),  j - bw <= i < j
//   Di[i] = 1 / U(i, i)
// and zero at every other position of a column (buffers cleared at setup).
// NR covers the bandwidth class of the factorisation window plus one block
// of 32 rows: R >= bw + 32.
// Window classes: up to 160 for every factorisation; 161..175 for the
// vector-unit one only (the blocked ones need 16 more than the bandwidth in a
// workgroup of at most 1024 threads).
constexpr int LU_MAX_BW = 175;
constexpr int lu_window_bw(int bw) {
    return bw <= 64 ? 64 : bw <= 96 ? 96 : bw <= 128 ? 128 : bw <= 160 ? 160 : bw <= LU_MAX_BW ? 176 : bw;
}
constexpr int solve_nr(int maxbw) { return lu_window_bw(maxbw) <= 176 ? (lu_window_bw(maxbw) + 32 + 63) / 64 : 0; }
__host__ __device__ inline int fac_pos(int s, int nr) {
    const int h = s >> 5;
    return ((s & 31) | ((h & 1) << 5)) * nr + (h >> 1);
}

template <typename T>
struct BandArgs {
    const BandSys *sys;
    const T *band;                // input band (read only)
    T *fac;                       // factors (offsets foff, lane-grouped slot-rotated layout)
    int *flags;
    const int *skip;
    T *dummy;                     // LU_DUMMY_PER_SYS elements per system: sink for masked stores
    const T *zero;                // a device zero, read by masked prefetches
    const T *one;                 // a device one (identity padding beyond n)
    // pivot and growth monitor (may be null): run-long maxima, as float bits,
    // of the growth factor max|u_ij| / max|a_ij| of a system and of
    // max|a_ij| / min|u_kk| (the inverse of its smallest relative pivot)
    float *stat = nullptr;
};

constexpr long long LU_DUMMY_PER_SYS = 1024;
// A pivot is too small when |u_kk| <= lu_tiny(T) * max|a_ij| of its system:
// below one rounding unit of the largest entry, where a pivot formed by
// cancellation keeps no correct digit.  (Pivots well below max|a_ij| are
// normal here: the pressure rows of the saddle-point systems eliminate to a
// Schur complement on a smaller scale.)  The growth is too large when
// max|u_ij| / max|a_ij| > lu_growth_limit(T): the factor's rounding, eps
// times the growth, would leave the refinement less than 2^-7 per sweep.
// Either raises flag bit 2.
template <typename T> constexpr float lu_tiny() { return sizeof(T) == 4 ? 0x1p-23f : 0x1p-52f; }
template <typename T> constexpr float lu_growth_limit() { return sizeof(T) == 4 ? 0x1p16f : 0x1p45f; }

template <typename T>
struct SolveArgs {
    const BandSys *sys;
    const T *fac;
    const double *r;
    double *x;
    const int *conv;
    int rhs_per_sys;
    const int *skip;
    const T *zero;                // device constants read by masked prefetches
    const T *one;
    const double *zero64;
    int assign = 0;               // 1: x = d (no prior x read), 0: x += d
};

struct DenseArgs {
    const double *inv;            // nsys column-major n x n inverses
    const double *b;              // nsys vectors of length n
    double *x;                    // x_s = inv_s b_s
    int n;
    const int *skip;
};

struct MergeArgs {
    const SysDesc *sys;           // the region's subdomains (x fastest)
    int nsx, N, region;
    const int32_t *own2_lo[2], *own2_n[2], *own1_lo[2], *own1_n[2];
    const double *base[3];
    const double *base1;
    const double *e2;
    const double *e1;
    double *out[3];
    double *out1;
    int nper = 0;                 // systems of the region per sample
    long long zs = 0;             // arena stride of base / out between samples (grid z = sample)
    const int8_t *cls2 = nullptr; // launch_lag_merged: local P2 node classes
    double *e2w = nullptr;        // launch_lag_merged: the corrections it rewrites (e2's buffer)
};

struct InitArgs {
    const SysDesc *sys;
    const int8_t *cls2;
    const double *ex[3];
    const double *pro[3];
    double *e;
    double *e1;
};

struct NewtonArgs {
    double *U;                    // U, P, e, e1: sample 0's in the per-sample arena
    double *P;
    const double *e;
    const double *e1;
    long long nu, np;
    int *done;                    // per sample
    int *its;                     // two per sample
    double tol;
    long long zs = 0;             // arena stride between samples
};

struct DenseNewtonArgs {
    DenseArgs d;                  // one system per sample: x = J^-1 b
    FinalizeArgs f;               // x to e_new, e_new1
    NewtonArgs u;                 // the update and its convergence test
    int *ticket;                  // blocks finished, per sample (reset by the last)
};

struct DensePorousArgs {
    DenseArgs d;                  // the three porous fields of one system per sample
    FinalizeArgs f;
    int *ticket;                  // per sample
};

struct NewtonStartArgs {
    const double *U0, *P0;        // level n
    const double *Um, *Pm;        // level n-1 (null at the first step)
    const double *Umm, *Pmm;      // level n-2 (null at the first two steps)
    double *U1, *P1;              // first iterate for level n+1
    long long nu2, np;
    int *done, *its;              // per sample (one, two)
    double *band;                 // the Jacobian band, cleared for its assembly (or null)
    long long band_n;
    int *flags;                   // bit 1 set if the previous coarse step ended unconverged
    long long zs = 0;             // arena stride between samples (grid row = sample)
};

// Restarted flexible GMRES over a batch of systems (krylov.hip).  Vectors are
// in the batch's vector space (system s at sys[s].dof_off, ntot entries per
// vector): V holds m + 1 basis vectors, Z the m preconditioned ones.  Per
// system: the Hessenberg matrix (m + 1) x m column-major, the Givens
// rotations, g, ||b||, a done flag and the steps taken.
constexpr int GM_MAX = 64;                          // largest restart length
constexpr size_t GM_LDS_MAX = 144 * 1024;           // Arnoldi work vector in LDS
struct GmresArgs {
    const SysDesc *sys;
    int m;
    long long ntot;
    double *V, *Z;
    double *H, *cs, *sn, *g, *bnorm;
    int *done, *kdone;
    double tol;                   // stop when |g_{k+1}| <= tol ||b||
    const int *conv;              // systems already converged (skipped), or null
    int *tot;                     // Arnoldi steps per system over the cycles of a local step
    int reorth;                   // 1: classical Gram-Schmidt with a second pass
};

// Restricted additive Schwarz over strips: strip vectors rs (right-hand
// sides) and zs (solutions) in the strip vector space.
struct StripArgs {
    const SysDesc *strip;
    const int32_t *parent;
    const SysDesc *sys;           // parent systems
    const int32_t *smap;
    const int8_t *sown;
    const int *done;              // parent done flags
    int *sdone;                   // per strip: skip (set by the gather)
    double *rs, *zs;
};

// first: the first cycle of a local step (clears the step's Arnoldi count)
bool launch_gm_init(const GmresArgs &a, int nsys, const double *r, const double *b, bool first, hipStream_t st);
// false if a system does not fit the LDS work vector or k is out of range
bool launch_gm_arnoldi(const GmresArgs &a, int nsys, int maxn, int k, const double *wneg, hipStream_t st);
void launch_gm_update(const GmresArgs &a, int nsys, double *x, hipStream_t st);
void launch_strip_gather(const StripArgs &a, int nstrip, const double *v, hipStream_t st);
void launch_strip_scatter(const StripArgs &a, int nstrip, double *z, hipStream_t st);
size_t gm_arnoldi_lds(int maxn);
void launch_fill_pattern(double *x, long long n, hipStream_t st);

hipError_t upload_constants(const RefData &r, hipStream_t st);
void launch_prolong_p2(const ProlongArgs &a, int nsamples, hipStream_t st);
void launch_prolong_p1(const ProlongArgs &a, int nsamples, hipStream_t st);
// Node-gather kernels run gridDim = (node blocks of GB threads, systems);
// maxnodes is the largest local P2 lattice of the batch.
constexpr int GB = 128;
int node_blocks(int maxnodes);
void launch_porous_rhs(const PorousArgs &a, int nsys, int maxnodes, int split, hipStream_t st);   // split 1 or 8 lanes per node
void launch_porous_finalize(const FinalizeArgs &a, int nsys, int maxnodes, hipStream_t st);
template <typename T>
void launch_porous_assemble(const AssembleArgs<T> &a, int nsys, hipStream_t st);
// split: lanes per node (1, or 8 for small problems: one lane per adjacent triangle)
void launch_oseen_rhs(const OseenArgs &a, int nsys, int maxnodes, int split, hipStream_t st);
template <typename T>
void launch_oseen_assemble(const OseenApplyArgs<T> &a, int nsys, int maxnodes, hipStream_t st);
// the same band entries as launch_oseen_assemble, one wavefront per lattice
// node, whole rows stored (no clearing needed); LDS 3 (2 maxbw + 1) entries
template <typename T>
void launch_oseen_rows(const OseenApplyArgs<T> &a, int nsys, int maxnodes, int maxbw, hipStream_t st);
// the same residual by tiles of 8 x 8 cells (each triangle integrated once);
// maxtiles = max over the systems of residual_tiles(cx, cy); its norm partials
// take 2 maxtiles doubles per system
int residual_tiles(int cx, int cy);
// blocks the residual launches aim for: each block beyond a box's first ends
// with a device-scope fence and ticket, so fewer, fuller blocks (measured at
// cfg2: 0.813 ms per step with two blocks per box, 0.826 with one, 0.87 with
// four)
constexpr long long RESIDUAL_BLOCKS_TARGET = 128;
void launch_oseen_residual_tiled(const OseenApplyArgs<double> &a, int nsys, int maxtiles, hipStream_t st);
// local Oseen right-hand sides by the same tiles
void launch_oseen_rhs_tiled(const OseenArgs &a, int nsys, int maxtiles, hipStream_t st);
// porous residuals (three fields) by the same tiles; partials as the Oseen one
void launch_porous_residual_tiled(const ResidualArgs &a, int nsys, int maxtiles, hipStream_t st);
// local porous right-hand sides by the same tiles
void launch_porous_rhs_tiled(const PorousArgs &a, int nsys, int maxtiles, hipStream_t st);
void launch_oseen_finalize(const FinalizeArgs &a, int nsys, int maxnodes, hipStream_t st);
template <typename T>
bool launch_band_lu(const BandArgs<T> &a, int nsys, int maxbw, int variant, hipStream_t st);
template <typename T>
bool launch_band_solve(const SolveArgs<T> &a, int nsys, int nrhs, int maxbw, int maxn, int depth, hipStream_t st);
void launch_dense_apply(const DenseArgs &a, int nsys, hipStream_t st);
void launch_merge(const MergeArgs &porous, const MergeArgs &conduit, int nsamples, hipStream_t st);   // both regions, every sample, one launch
// after launch_merge: every subdomain's porous and velocity corrections
// replaced by the merged correction out - base on its local lattice (zero on
// artificial nodes), the lagged e^n of LP_LAG_MERGED
void launch_lag_merged(const MergeArgs &porous, const MergeArgs &conduit, int nsamples, hipStream_t st);
void launch_init_corrections(const InitArgs &a, int nsys, hipStream_t st);
void launch_newton_update(const NewtonArgs &a, int nsamples, hipStream_t st);
void launch_dense_newton(const DenseNewtonArgs &a, int nsamples, hipStream_t st);
void launch_dense_porous(const DensePorousArgs &a, int nsys, hipStream_t st);   // nsys = 3 per sample
void launch_newton_start(const NewtonStartArgs &a, int nsamples, hipStream_t st);
// The time level of a step on the device: m = *level, then *level = m + stride,
// t = m dt (a product, never accumulated) and tf = (cos t, sin t, cos^2 t).
// Each ring slot has its own counter, advanced by the ring's size, so every
// replay of a step's launches reads the time of its own level.
void launch_time_level(long long *level, long long stride, double dt, double *tf, hipStream_t st);
// p[0..n) = 0 by a small kernel (capturable in a graph, unlike a memset node)
void launch_zero_ints(int *p, long long n, hipStream_t st);
// bytes of p (a 16-byte aligned device buffer) set to zero by a kernel
void launch_zero_fill(void *p, size_t bytes, hipStream_t st);

}  // namespace lp
