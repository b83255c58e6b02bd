// HIP kernels of the local parallel stage (gfx950).
//
// Every local problem lives on a box of one grid (a subdomain Omega_j of T_h,
// or a whole region of T_H for the coarse step).  Element work never scatters:
// either a node gathers its rows from the (at most six) triangles around it
// (one thread per node for the band assembly, eight lanes per node or one
// wavefront per node on the single coarse system), or a workgroup integrates
// the triangles of a tile of cells once into LDS and its node threads gather
// from there (the local right-hand sides and residuals).  A node always adds
// its triangles in the same order, so results are deterministic without
// atomics.  Linear systems are banded (lattice-row ordering) and factored
// without pivoting by one workgroup per system with the active window held in
// registers; triangular solves run one wavefront per right-hand side.
#include <hip/hip_runtime.h>
#include <type_traits>
#include <utility>
#include <cmath>

#include "kernels.h"

namespace lp {

__constant__ RefData c_ref;

hipError_t upload_constants(const RefData &r, hipStream_t st) {
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_ref), &r, sizeof(RefData), 0, hipMemcpyHostToDevice, st);
}

// ---------------------------------------------------------------------------
// element helpers
// ---------------------------------------------------------------------------
// local index (0..5) of the P2 node at in-cell half coordinates (la, lb) in
// orientation t, or -1 if the node is not on that triangle
__device__ __forceinline__ int p2_local(int t, int la, int lb) {
    if (t == 0) {
        if (la < lb) return -1;
        const int tab[3][3] = {{0, -1, -1}, {3, 5, -1}, {1, 4, 2}};   // [la][lb]
        return tab[la][lb];
    } else {
        if (la > lb) return -1;
        const int tab[3][3] = {{0, 5, 2}, {-1, 3, 4}, {-1, -1, 1}};
        return tab[la][lb];
    }
}

// P1 local index of the vertex at in-cell vertex coordinates (i, j)
__device__ __forceinline__ int p1_local(int t, int i, int j) {
    if (t == 0) { if (i == 0 && j == 0) return 0; if (i == 1 && j == 0) return 1; if (i == 1 && j == 1) return 2; return -1; }
    if (i == 0 && j == 0) return 0; if (i == 1 && j == 1) return 1; if (i == 0 && j == 1) return 2; return -1;
}

// Visit the triangles of a box (cx x cy cells) containing the box-local P2
// node (a, b): f(t, ci, cj, la) with box-local cell indices.
template <class F>
__device__ __forceinline__ void for_elements(int a, int b, int cx, int cy, F &&f) {
    const int ci0 = (a - 1) >> 1 < 0 ? 0 : ((a - 1) >> 1);
    const int ci1 = (a >> 1) < cx ? (a >> 1) : cx - 1;
    const int cj0 = (b - 1) >> 1 < 0 ? 0 : ((b - 1) >> 1);
    const int cj1 = (b >> 1) < cy ? (b >> 1) : cy - 1;
    for (int cj = cj0; cj <= cj1; ++cj)
        for (int ci = ci0; ci <= ci1; ++ci) {
            const int la = a - 2 * ci, lb = b - 2 * cj;
            if (la < 0 || la > 2 || lb < 0 || lb > 2) continue;
            for (int t = 0; t < 2; ++t) {
                const int k = p2_local(t, la, lb);
                if (k >= 0) f(t, ci, cj, k);
            }
        }
}

// ---------------------------------------------------------------------------
// Prolongation Pi_h (exact evaluation of coarse P2 / P1 functions at fine nodes)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void p2_values(double xi, double eta, double v[6]) {
    const double l0 = 1.0 - xi - eta, l1 = xi, l2 = eta;
    v[0] = l0 * (2 * l0 - 1); v[1] = l1 * (2 * l1 - 1); v[2] = l2 * (2 * l2 - 1);
    v[3] = 4 * l0 * l1; v[4] = 4 * l1 * l2; v[5] = 4 * l0 * l2;
}

// A latency-bound kernel claims the whole register file of each SIMD it runs
// on (v255 and a255 count as used, 512 registers), so no wavefront of the
// concurrent streams shares its instruction issue.  Only for workgroups of at
// most four wavefronts (one per SIMD of the compute unit): a workgroup of more
// wavefronts with this allocation cannot be dispatched (the queue aborts with
// an invalid-code-object error).  The caller passes its launch bound, which
// must be the same constant as in its __launch_bounds__, and the bound is
// checked at compile time.
template <int BLOCK_THREADS>
__device__ __forceinline__ void own_simd() {
    static_assert(BLOCK_THREADS <= 256, "own_simd: a full register claim needs workgroups of at most four wavefronts");
    asm volatile("" ::: "v255", "a255");
}

__global__ void k_prolong_p2(ProlongArgs A) {
    const long long zo = blockIdx.y * A.zs;
    const int nf = 2 * A.Nh + 1, nc = 2 * A.NH + 1;
    const long long tot = (long long)nf * nf;
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < tot; g += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(g % nf), b = (int)(g / nf);
        const int k2 = 2 * A.k;                    // fine half-steps per coarse cell
        int ci = a / k2, cj = b / k2;
        if (ci >= A.NH) ci = A.NH - 1;
        if (cj >= A.NH) cj = A.NH - 1;
        const int la = a - k2 * ci, lb = b - k2 * cj;   // 0..k2
        const double lx = (double)la / k2, ly = (double)lb / k2;
        const int t = lb > la ? 1 : 0;
        double xi, eta;
        if (t == 0) { xi = lx - ly; eta = ly; } else { xi = lx; eta = ly - lx; }
        double v[6];
        p2_values(xi, eta, v);
        for (int f = 0; f < A.nfields; ++f) {
            const double *src = A.src[f] + zo;
            double s = 0.0;
            for (int q = 0; q < 6; ++q)
                s += v[q] * src[(2 * ci + off2a(t, q)) + (long long)nc * (2 * cj + off2b(t, q))];
            A.dst[f][zo + g] = s;
        }
    }
}

__global__ void k_prolong_p1(ProlongArgs A) {
    const long long zo = blockIdx.y * A.zs;
    const int nf = A.Nh + 1, nc = A.NH + 1;
    const long long tot = (long long)nf * nf;
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < tot; g += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(g % nf), j = (int)(g / nf);
        int ci = i / A.k, cj = j / A.k;
        if (ci >= A.NH) ci = A.NH - 1;
        if (cj >= A.NH) cj = A.NH - 1;
        const double lx = (double)(i - A.k * ci) / A.k, ly = (double)(j - A.k * cj) / A.k;
        const int t = (j - A.k * cj) > (i - A.k * ci) ? 1 : 0;
        double l[3];
        if (t == 0) { l[1] = lx - ly; l[2] = ly; } else { l[1] = lx; l[2] = ly - lx; }
        l[0] = 1.0 - l[1] - l[2];
        for (int f = 0; f < A.nfields; ++f) {
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += l[q] * A.src[f][zo + (ci + off1a(t, q)) + (long long)nc * (cj + off1b(t, q))];
            A.dst[f][zo + g] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Porous systems (Eqs. (5.1)-(5.3) on T_H, (5.5)-(5.7) on Omega_j)
//   A_f = (tau_f + x_f) M + kap_f K,  x_F = s*, x_f = s + s*, x_m = s
//   b_f = Q_f + M[tau_f (O_f - X_f) - x_f X_f + sum_k c_fk O_k] - kap_f K X_f + Gamma_f
//   X_f = P_f^{n+1} + z_f (background at n+1 plus Dirichlet values of the correction),
//   O_f = P_f^n + e_f^n (background at n plus the previous correction).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double porous_x(const Coef &cf, int f) { return f == 0 ? cf.sst : f == 1 ? cf.s + cf.sst : cf.s; }

// Dirichlet value of field f of the correction at local P2 node q of system S
__device__ __forceinline__ double porous_z(const SysDesc &S, const PorousArgs &A, int f, int q, long long G) {
    const int c = A.cls2[S.node_off + q];
    if (c != 1) return 0.0;
    const double bg = A.P1[f] ? A.P1[f][S.zo + G] : 0.0;
    return A.ex[f][G] * A.tf[0] - bg;
}

// The e-th triangle (e = 0..5) around box-local P2 node (a, b), in the order
// for_elements visits them; false if the node has fewer.
__device__ __forceinline__ bool nth_element(int a, int b, int cx, int cy, int e, int &t_, int &ci_, int &cj_, int &la_) {
    const int ci0 = (a - 1) >> 1 < 0 ? 0 : ((a - 1) >> 1);
    const int ci1 = (a >> 1) < cx ? (a >> 1) : cx - 1;
    const int cj0 = (b - 1) >> 1 < 0 ? 0 : ((b - 1) >> 1);
    const int cj1 = (b >> 1) < cy ? (b >> 1) : cy - 1;
    int cnt = 0;
    bool found = false;
    for (int cj = cj0; cj <= cj1; ++cj)
        for (int ci = ci0; ci <= ci1; ++ci) {
            const int la = a - 2 * ci, lb = b - 2 * cj;
            if (la < 0 || la > 2 || lb < 0 || lb > 2) continue;
            for (int t = 0; t < 2; ++t) {
                const int k = p2_local(t, la, lb);
                if (k >= 0) {
                    if (cnt == e) { t_ = t; ci_ = ci; cj_ = cj; la_ = k; found = true; }
                    ++cnt;
                }
            }
        }
    return found;
}

// sum over the SPLIT consecutive lanes of a node group
template <int SPLIT>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = SPLIT / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, SPLIT);
    return v;
}

// SPLIT = 1: one thread per node walks the node's triangles.  SPLIT = 8: eight
// lanes per node, lane e takes the e-th triangle and the group adds up (the
// single coarse system, where a thread per node leaves the chip idle).
template <int SPLIT>
__global__ __launch_bounds__(GB) void k_porous_rhs(PorousArgs A) {
    static_assert(GB % SPLIT == 0, "node groups within a block");
    const SysDesc S = A.sys[blockIdx.y];
    const Coef &cf = A.co[S.sample];   // the coefficients of the system's sample
    const int nloc = S.lw2 * S.lh2;
    const int ng = 2 * S.N + 1;
    const double h = S.h, h2 = h * h;
    const int sub = SPLIT > 1 ? (int)(threadIdx.x % SPLIT) : 0;
    for (int qq = blockIdx.x * GB + threadIdx.x; qq < nloc * SPLIT; qq += gridDim.x * GB) {
        const int q = qq / SPLIT;
        const int a = q % S.lw2, b = q / S.lw2;
        const long long G = (2 * S.x0 + a) + (long long)ng * (2 * S.y0 + b);
        const int cls = A.cls2[S.node_off + q];
        if (cls != 0) {
            if (sub == 0)
                for (int f = 0; f < 3; ++f) A.e_new[S.e2_off + (long long)f * nloc + q] = porous_z(S, A, f, q, G);
            continue;
        }
        // sources at t_{n+1}; the three fields together, so each node of a
        // triangle is read once for all of them
        double r[3];
        for (int f = 0; f < 3; ++f) r[f] = sub == 0 ? A.load[f][0][S.zo + G] * A.tf[0] + A.load[f][1][S.zo + G] * A.tf[1] : 0.0;
        auto elem = [&](int t, int ci, int cj, int la) {
            double mv[3] = {0.0, 0.0, 0.0}, kv[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < 6; ++k) {
                const int qa = 2 * ci + off2a(t, k), qb = 2 * cj + off2b(t, k);
                const int qk = qa + S.lw2 * qb;
                const long long Gk = (2 * S.x0 + qa) + (long long)ng * (2 * S.y0 + qb);
                const bool dir = A.cls2[S.node_off + qk] == 1;
                double O[3], X[3];
                for (int g = 0; g < 3; ++g) {
                    const double p1 = A.P1[g] ? A.P1[g][S.zo + Gk] : 0.0;
                    O[g] = (A.P0[g] ? A.P0[g][S.zo + Gk] : 0.0) + A.e_old[S.e2_off + (long long)g * nloc + qk];
                    X[g] = p1 + (dir ? A.ex[g][Gk] * A.tf[0] - p1 : 0.0);
                }
                for (int f = 0; f < 3; ++f) {
                    double m = cf.tau[f] * (O[f] - X[f]) - porous_x(cf, f) * X[f];
                    if (f == 0) m += cf.sst * O[1];
                    if (f == 1) m += cf.s * O[2] + cf.sst * O[0];
                    if (f == 2) m += cf.s * O[1];
                    mv[f] += c_ref.Me[t][la][k] * m;
                    kv[f] += c_ref.Ke[t][la][k] * X[f];
                }
            }
            for (int f = 0; f < 3; ++f) r[f] += h2 * mv[f] - cf.kap[f] * kv[f];
        };
        if (SPLIT == 1) {
            for_elements(a, b, S.cx, S.cy, elem);
        } else {
            int t, ci, cj, la;
            if (nth_element(a, b, S.cx, S.cy, sub, t, ci, cj, la)) elem(t, ci, cj, la);
            // every lane of the group takes part (same node, same branch)
            for (int f = 0; f < 3; ++f) r[f] = group_sum<SPLIT>(r[f]);
            if (sub != 0) continue;
        }
        // + <u^n . n_c, v_F>_Gamma = -int_Gamma v_F u_y^n on the porous top row
        if (S.gamma && 2 * S.y0 + b == 2 * S.N && A.Uy0) {
            const int A0 = 2 * S.x0 + a;
            const int ne = (A0 & 1) ? 1 : 2;
            for (int e = 0; e < ne; ++e) {
                const int ie = (A0 & 1) ? (A0 >> 1) : (A0 >> 1) - 1 + e;
                if (ie < S.x0 || ie >= S.x0 + S.cx) continue;
                const int la = A0 - 2 * ie;
                double sg = 0.0;
                for (int k = 0; k < 3; ++k) sg += c_ref.Ge[la][k] * A.Uy0[S.zo + 2 * ie + k];   // conduit Gamma row b = 0
                r[0] -= h * sg;
            }
        }
        const int d = A.dof2[S.node_off + q];
        for (int f = 0; f < 3; ++f) A.b[S.dof_off + (long long)f * S.ndof + d] = r[f];
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Reduction of ||r||^2 and ||b||^2 of system `id` over the gridDim.x node
// blocks that share it.  Each block stores its partial sums; the block that
// arrives last (ticket counter) adds the partials in block order, so the
// result does not depend on scheduling, records the relative residual,
// counts the sweep, raises the convergence flag and rearms the counter.
__device__ void grid_norms_and_flag(double rr, double bb, double *part, int *ticket, int *conv, double *relres,
                                    int *sweeps, double tol, int id) {
    __shared__ double s1[16], s2[16];       // one per wavefront (blocks of up to 1024 threads)
    __shared__ int last;
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) { s1[w] = rr; s2[w] = bb; }
    __syncthreads();
    if (gridDim.x == 1) {
        // the whole system in this block: no partials, ticket or fence
        if (threadIdx.x == 0) {
            double a = 0.0, b = 0.0;
            for (int i = 0; i < nw; ++i) { a += s1[i]; b += s2[i]; }
            const double rel = b > 0.0 ? sqrt(a / b) : 0.0;
            relres[id] = rel;
            sweeps[id] += 1;
            if (rel <= tol) conv[id] = 1;
        }
        __syncthreads();                    // s1, s2 free for the next call
        return;
    }
    const long long base = 2LL * id * gridDim.x;
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < nw; ++i) { a += s1[i]; b += s2[i]; }
        part[base + 2 * blockIdx.x] = a;
        part[base + 2 * blockIdx.x + 1] = b;
        __threadfence();
        last = atomicAdd(ticket + id, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        double a = 0.0, b = 0.0;
        for (int i = 0; i < (int)gridDim.x; ++i) {
            a += part[base + 2 * i];
            b += part[base + 2 * i + 1];
        }
        ticket[id] = 0;
        const double rel = b > 0.0 ? sqrt(a / b) : 0.0;
        relres[id] = rel;
        sweeps[id] += 1;
        if (rel <= tol) conv[id] = 1;
    }
}

// Norms of the tiled residual kernels, in an order that does not depend on
// how many blocks share a box: each tile's sums of r^2 and b^2 are reduced in
// the block (wavefront sums, then the wavefronts in order), and the tiles'
// sums are added in tile order, by a running total when one block takes the
// whole box, else by the last of the box's blocks from the tiles' partials
// (part[2 ((id0 + f) tstride + tile)]).  tile_norms: after each tile;
// tile_norms_finish: after the last, by every thread of every block.
template <int F>
__device__ __forceinline__ void tile_norms(double (&r)[F], double (&b)[F], const bool (&act)[F], double (&tr)[F],
                                           double (&tb)[F], double *part, int tstride, int id0, int tile) {
    __shared__ double s[2 * F][16];
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const double x = wave_sum(r[f]), y = wave_sum(b[f]);
        if ((threadIdx.x & 63) == 0) { s[2 * f][w] = x; s[2 * f + 1][w] = y; }
    }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < F; ++f) {
        double x = 0.0, y = 0.0;
        for (int i = 0; i < nw; ++i) { x += s[2 * f][i]; y += s[2 * f + 1][i]; }
        if (gridDim.x == 1) {
            tr[f] += x;
            tb[f] += y;
        } else if (threadIdx.x == 0 && act[f]) {
            const long long at = 2 * ((long long)(id0 + f) * tstride + tile);
            part[at] = x;
            part[at + 1] = y;
        }
    }
    __syncthreads();                        // s free for the next tile
}
template <int F>
__device__ void tile_norms_finish(const double (&tr)[F], const double (&tb)[F], const bool (&act)[F], double *part,
                                  int *ticket, int *conv, double *relres, int *sweeps, double tol, int id0, int tstride,
                                  int ntile) {
    auto done = [&](int f, double a, double b) {
        const double rel = b > 0.0 ? sqrt(a / b) : 0.0;
        relres[id0 + f] = rel;
        sweeps[id0 + f] += 1;
        if (rel <= tol) conv[id0 + f] = 1;
    };
    if (gridDim.x == 1) {
        if (threadIdx.x == 0)
            for (int f = 0; f < F; ++f)
                if (act[f]) done(f, tr[f], tb[f]);
        return;
    }
    __shared__ int last;
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(ticket + id0, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        ticket[id0] = 0;
        for (int f = 0; f < F; ++f) {
            if (!act[f]) continue;
            double a = 0.0, b = 0.0;
            const long long base = 2LL * (id0 + f) * tstride;
            for (int t = 0; t < ntile; ++t) {
                a += part[base + 2 * t];
                b += part[base + 2 * t + 1];
            }
            done(f, a, b);
        }
    }
}

// y = A_f x restricted to free rows (FP64, matrix-free); r = b - y; norms
__device__ __forceinline__ void porous_finalize_rows(const FinalizeArgs &F, const SysDesc &S, int start, int stride) {
    const int nloc = S.lw2 * S.lh2;
    for (int q = start; q < nloc; q += stride) {
        const int d = F.dof2[S.node_off + q];
        if (d < 0) continue;
        for (int f = 0; f < 3; ++f)
            F.e_new[S.e2_off + (long long)f * nloc + q] = F.x[S.dof_off + (long long)f * S.ndof + d];
    }
}
// the first block of each system folds its refinement outcome into the run totals
__device__ __forceinline__ void record_ir_totals(const IrTotals &T) {
    if (!T.flags || blockIdx.x != 0 || (int)threadIdx.x >= T.ids_per_sys) return;
    const int id = blockIdx.y * T.ids_per_sys + threadIdx.x;
    if (!T.conv[id]) atomicOr(T.flags, 1);
    atomicMax(T.max_sweeps, T.sweeps[id]);
    atomicMax(T.max_relres, (unsigned long long)__double_as_longlong(T.relres[id]));
}

__global__ __launch_bounds__(GB) void k_porous_finalize(FinalizeArgs F) {
    const SysDesc S = F.sys[blockIdx.y];
    if (F.skip && F.skip[S.sample]) return;
    record_ir_totals(F.acc);
    porous_finalize_rows(F, S, blockIdx.x * GB + threadIdx.x, gridDim.x * GB);
}

// band assembly of the constant porous matrices (setup)
template <typename T>
__global__ __launch_bounds__(256) void k_porous_assemble(AssembleArgs<T> A) {
    const SysDesc S = A.sys[blockIdx.x];
    const Coef &cf = A.co[S.sample];   // the coefficients of the system's sample
    const int nloc = S.lw2 * S.lh2;
    const int ld = 2 * S.bw + 1;
    const double h2 = S.h * S.h;
    for (int q = threadIdx.x; q < nloc; q += blockDim.x) {
        const int dq = A.dof2[S.node_off + q];
        if (dq < 0) continue;
        const int a = q % S.lw2, bq = q / S.lw2;
        for (int f = 0; f < 3; ++f) {
            T *band = A.band + S.band_off + (long long)f * S.band_size;
            const double tau = cf.tau[f], xf = porous_x(cf, f), kap = cf.kap[f];
            for_elements(a, bq, S.cx, S.cy, [&](int t, int ci, int cj, int la) {
                for (int k = 0; k < 6; ++k) {
                    const int qk = (2 * ci + off2a(t, k)) + S.lw2 * (2 * cj + off2b(t, k));
                    const int dk = A.dof2[S.node_off + qk];
                    if (dk < 0) continue;
                    const double v = (tau + xf) * h2 * c_ref.Me[t][la][k] + kap * c_ref.Ke[t][la][k];
                    T *p = band + (long long)dk * ld + (dq - dk + S.bw);
                    *p = (T)((double)*p + v);
                }
            });
        }
    }
}

// ---------------------------------------------------------------------------
// Oseen systems (Eq. (5.4) linearised by Newton on T_H, Eq. (5.8) on Omega_j)
//   [eta/dt M + nu eta S + eta beta G_Gamma + eta N(W)] e - eta B^T d = b_u
//   eta B e = b_q
// ---------------------------------------------------------------------------
// element values of the box-local velocity nodes of triangle (t, ci, cj)
struct ElemVel {
    double w[2][6];      // background W^{n+1}
};

// velocity Dirichlet value of the correction at local node q
__device__ __forceinline__ double oseen_z(const SysDesc &S, const OseenArgs &A, int c, int q, long long G) {
    if (A.cls2[S.node_off + q] != 1) return 0.0;
    return A.ex[c][G] * A.tf[0] - A.W1[c][S.zo + G];
}

// convection rows at test node la of triangle t (unit-cell reference data,
// scaled by h): cW[c] = int ((W.grad)W)_c phi_la, Nz[c] = int (N(W) z)_c phi_la
__device__ __forceinline__ void conv_rows(int t, int la, double h, const double W[2][6], const double Z[2][6],
                                          bool want_c, double cW[2], double Nz[2]) {
    cW[0] = cW[1] = Nz[0] = Nz[1] = 0.0;
    // Reference values are read at uniform addresses (scalar loads) and the
    // lane picks its orientation and test node from them: indexing by the
    // per-lane t or la would turn every read into a vector memory access.
#pragma unroll 2
    for (int q = 0; q < NQ; ++q) {
        double wv[2] = {0, 0}, gw[2][2] = {{0, 0}, {0, 0}}, zv[2] = {0, 0}, gz[2][2] = {{0, 0}, {0, 0}};
        double pla = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double p = c_ref.phi[q][k];
            const double dx0 = c_ref.dphi[0][q][k][0], dx1 = c_ref.dphi[1][q][k][0];
            const double dy0 = c_ref.dphi[0][q][k][1], dy1 = c_ref.dphi[1][q][k][1];
            const double dx = t ? dx1 : dx0, dy = t ? dy1 : dy0;
            pla = la == k ? p : pla;
            for (int c = 0; c < 2; ++c) {
                wv[c] += W[c][k] * p;
                gw[c][0] += W[c][k] * dx;
                gw[c][1] += W[c][k] * dy;
                zv[c] += Z[c][k] * p;
                gz[c][0] += Z[c][k] * dx;
                gz[c][1] += Z[c][k] * dy;
            }
        }
        const double wt = c_ref.w[q] * pla;
        for (int c = 0; c < 2; ++c) {
            if (want_c) cW[c] += wt * (wv[0] * gw[c][0] + wv[1] * gw[c][1]);
            Nz[c] += wt * (zv[0] * gw[c][0] + zv[1] * gw[c][1] + wv[0] * gz[c][0] + wv[1] * gz[c][1]);
        }
    }
    // h^2 (area) * 1/h (one derivative)
    for (int c = 0; c < 2; ++c) { cW[c] *= h; Nz[c] *= h; }
}


// SPLIT = 1: one thread per node walks the node's triangles.  SPLIT = 8: eight
// lanes per node, lane e takes the e-th triangle and the group adds up (for
// the small coarse problem, where a thread per node leaves the chip idle and
// the per-node work is the latency).
template <int SPLIT>
__global__ __launch_bounds__(GB) void k_oseen_rhs(OseenArgs A) {
    static_assert(GB % SPLIT == 0, "node groups within a block");
    const SysDesc S = A.sys[blockIdx.y];
    const Coef &cf = A.co[S.sample];   // the coefficients of the system's sample
    if (A.skip && A.skip[S.sample]) return;
    const int nloc = S.lw2 * S.lh2;
    const int ng = 2 * S.N + 1, ng1 = S.N + 1;
    const double h = S.h, h2 = h * h;
    const double eta = cf.eta, edt = cf.eta / cf.dt, nue = cf.nu * cf.eta;
    const int sub = SPLIT > 1 ? (int)(threadIdx.x % SPLIT) : 0;
    for (int qq = blockIdx.x * GB + threadIdx.x; qq < nloc * SPLIT; qq += gridDim.x * GB) {
        const int q = qq / SPLIT;
        const int a = q % S.lw2, b = q / S.lw2;
        const long long G = (2 * S.x0 + a) + (long long)ng * (2 * S.y0 + b);
        const int cls = A.cls2[S.node_off + q];
        double *en = A.e_new + S.e2_off;
        const bool vertex = !(a & 1) && !(b & 1);
        const int vq = vertex ? (a >> 1) + S.lw1 * (b >> 1) : -1;
        const bool prow = vertex && A.cls1[S.vert_off + vq] == 0;
        if (sub == 0) {
            if (cls != 0)
                for (int c = 0; c < 2; ++c) en[(long long)c * nloc + q] = oseen_z(S, A, c, q, G);
            if (vertex && !prow) A.e_new1[S.e1_off + vq] = 0.0;
        }
        const bool active = cls == 0 || prow;
        double rv[2] = {0.0, 0.0}, rq = 0.0;
        if (active && cls == 0 && sub == 0)
            for (int c = 0; c < 2; ++c)
                rv[c] = eta * (A.load[c][0][S.zo + G] * A.tf[0] + A.load[c][1][S.zo + G] * A.tf[1] + A.load[c][2][S.zo + G] * A.tf[2]);
        auto elem = [&](int t, int ci, int cj, int la) {
            double W[2][6], Z[2][6], Y[2][6], O[2][6], P[3];
            for (int k = 0; k < 6; ++k) {
                const int qa = 2 * ci + off2a(t, k), qb = 2 * cj + off2b(t, k);
                const int qk = qa + S.lw2 * qb;
                const long long Gk = (2 * S.x0 + qa) + (long long)ng * (2 * S.y0 + qb);
                for (int c = 0; c < 2; ++c) {
                    W[c][k] = A.W1[c][S.zo + Gk];
                    Z[c][k] = oseen_z(S, A, c, qk, Gk);
                    Y[c][k] = W[c][k] + Z[c][k];
                    O[c][k] = (A.W0[c] ? A.W0[c][S.zo + Gk] : 0.0) + (A.e_old ? A.e_old[S.e2_off + (long long)c * nloc + qk] : 0.0)
                              - W[c][k] - Z[c][k];
                }
            }
            for (int k = 0; k < 3; ++k)
                P[k] = A.Pp[S.zo + (S.x0 + ci + off1a(t, k)) + (long long)ng1 * (S.y0 + cj + off1b(t, k))];
            if (cls == 0) {
                double cW[2], Nz[2];
                if (cf.convection) conv_rows(t, la, h, W, Z, true, cW, Nz);
                else cW[0] = cW[1] = Nz[0] = Nz[1] = 0.0;
                for (int c = 0; c < 2; ++c) {
                    double m = 0.0, sv = 0.0, bt = 0.0;
                    for (int k = 0; k < 6; ++k) {
                        m += c_ref.Me[t][la][k] * O[c][k];
                        for (int d = 0; d < 2; ++d) sv += c_ref.Se[t][c * 6 + la][d * 6 + k] * Y[d][k];
                    }
                    for (int v = 0; v < 3; ++v) bt += c_ref.Be[t][v][c * 6 + la] * P[v];
                    rv[c] += edt * h2 * m - nue * sv - eta * (cW[c] + Nz[c]) + eta * h * bt;
                }
            }
            if (prow) {
                const int lv = p1_local(t, (a >> 1) - ci, (b >> 1) - cj);
                double sv = 0.0;
                for (int d = 0; d < 2; ++d)
                    for (int k = 0; k < 6; ++k) sv += c_ref.Be[t][lv][d * 6 + k] * Y[d][k];
                rq -= eta * h * sv;
            }
        };
        if (active) {
            if (SPLIT == 1) {
                for_elements(a, b, S.cx, S.cy, elem);
            } else {
                int t, ci, cj, la;
                if (nth_element(a, b, S.cx, S.cy, sub, t, ci, cj, la)) elem(t, ci, cj, la);
            }
        }
        if (SPLIT > 1) {
            // every lane of the group takes part (same node, same branch)
            rv[0] = group_sum<SPLIT>(rv[0]);
            rv[1] = group_sum<SPLIT>(rv[1]);
            rq = group_sum<SPLIT>(rq);
        }
        if (!active || sub != 0) continue;
        // Gamma edges (conduit bottom row): Beavers-Joseph on the x rows and the
        // lagged p_F^n terms -(eta/rho) int p_F v.n_c - c_tau int d_x p_F v_x
        if (cls == 0 && S.gamma && 2 * S.y0 + b == 0) {
            const int A0 = 2 * S.x0 + a;
            const int ne = (A0 & 1) ? 1 : 2;
            for (int e = 0; e < ne; ++e) {
                const int ie = (A0 & 1) ? (A0 >> 1) : (A0 >> 1) - 1 + e;
                if (ie < S.x0 || ie >= S.x0 + S.cx) continue;
                const int la = A0 - 2 * ie;
                double bj = 0.0, pg = 0.0, pgx = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const int qk = (2 * ie + k - 2 * S.x0);     // box-local, row 0
                    const long long Gk = 2 * ie + k;           // grid conduit row 0
                    bj += c_ref.Ge[la][k] * (A.W1[0][S.zo + Gk] + oseen_z(S, A, 0, qk, Gk));
                    const double pf = A.PF0[S.zo + (2 * ie + k) + (long long)ng * (2 * S.N)];   // porous top row
                    pg += c_ref.Ge[la][k] * pf;
                    pgx += c_ref.Gxe[la][k] * pf;
                }
                rv[0] -= eta * cf.beta * h * bj + cf.ctau * pgx;
                rv[1] += eta / cf.rho * h * pg;
            }
        }
        if (cls == 0) {
            const int d = A.dof2[S.node_off + q];
            A.b[S.dof_off + d] = rv[0];
            A.b[S.dof_off + d + 1] = rv[1];
        }
        if (prow) A.b[S.dof_off + A.dof1[S.vert_off + vq]] = rq;
    }
}

// Band assembly of the local Oseen operators (T), one thread per node: its
// rows, added element by element.  With first_write the band was cleared
// once, at setup: the matrices' pattern is the same every step, so entries
// outside it are still zero, and an entry's first element stores its value
// (0 + v, the same rounding as adding to the cleared entry) instead of
// reading the entry back; masks over the node's 5 x 5 lattice neighbourhood
// record the column nodes earlier elements have touched.  Without it the
// band is cleared before every assembly and every entry is read back.
template <typename T>
__global__ __launch_bounds__(GB) void k_oseen_assemble(OseenApplyArgs<T> A) {
    const SysDesc S = A.sys[blockIdx.y];
    const Coef &cf = A.co[S.sample];   // the coefficients of the system's sample
    if (A.skip && A.skip[S.sample]) return;
    const int nloc = S.lw2 * S.lh2;
    const int ng = 2 * S.N + 1;
    const double h = S.h, h2 = h * h;
    const double eta = cf.eta, edt = cf.eta / cf.dt, nue = cf.nu * cf.eta;
    const int ld = 2 * S.bw + 1;
    T *band = A.band + S.band_off;
    auto put = [&](int row, int col, double v) {
        T *p = band + (long long)col * ld + (row - col + S.bw);
        *p = (T)((double)*p + v);
    };
    const bool fw = A.first_write != 0;
    for (int q = blockIdx.x * GB + threadIdx.x; q < nloc; q += gridDim.x * GB) {
        const int a = q % S.lw2, b = q / S.lw2;
        const int cls = A.cls2[S.node_off + q];
        const bool vertex = !(a & 1) && !(b & 1);
        const int vq = vertex ? (a >> 1) + S.lw1 * (b >> 1) : -1;
        const int dv = cls == 0 ? A.dof2[S.node_off + q] : -1;
        const int dp = vertex ? A.dof1[S.vert_off + vq] : -1;
        if (dv < 0 && dp < 0) continue;
        // column nodes (velocity) and vertices (pressure) touched so far, bit
        // (qa - a + 2) + 5 (qb - b + 2) of lattice node (qa, qb)
        unsigned seen_v = 0u, seen_p = 0u;
        auto nbit = [&](int qa, int qb) { return 1u << ((qa - a + 2) + 5 * (qb - b + 2)); };
        for_elements(a, b, S.cx, S.cy, [&](int t, int ci, int cj, int la) {
            // bit k of fv / fp: column node / vertex k first met in this element
            unsigned fv = 0u, fp = 0u;
            if (fw) {
                for (int k = 0; k < 6; ++k) {
                    const unsigned bit = nbit(2 * ci + off2a(t, k), 2 * cj + off2b(t, k));
                    if (!(seen_v & bit)) fv |= 1u << k;
                    seen_v |= bit;
                }
                for (int k = 0; k < 3; ++k) {
                    const unsigned bit = nbit(2 * (ci + off1a(t, k)), 2 * (cj + off1b(t, k)));
                    if (!(seen_p & bit)) fp |= 1u << k;
                    seen_p |= bit;
                }
            }
            double W[2][6];
            int dk[6], pk[3];
            for (int k = 0; k < 6; ++k) {
                const int qa = 2 * ci + off2a(t, k), qb = 2 * cj + off2b(t, k);
                const int qk = qa + S.lw2 * qb;
                const long long Gk = (2 * S.x0 + qa) + (long long)ng * (2 * S.y0 + qb);
                dk[k] = A.dof2[S.node_off + qk];
                for (int c = 0; c < 2; ++c) W[c][k] = A.W1[c][S.zo + Gk];
            }
            for (int k = 0; k < 3; ++k)
                pk[k] = A.dof1[S.vert_off + (ci + off1a(t, k)) + S.lw1 * (cj + off1b(t, k))];
            if (dv >= 0) {
                {
                    // entries of rows (la, c) against columns (k, d) and pressure v
                    double Nw[2][2][6];     // [c][d][k]
                    for (int c = 0; c < 2; ++c) for (int d = 0; d < 2; ++d) for (int k = 0; k < 6; ++k) Nw[c][d][k] = 0.0;
                    if (cf.convection && !A.no_convection) {
                        for (int qq = 0; qq < NQ; ++qq) {
                            double wv[2] = {0, 0}, gw[2][2] = {{0, 0}, {0, 0}};
                            for (int k = 0; k < 6; ++k) {
                                const double p = c_ref.phi[qq][k];
                                for (int c = 0; c < 2; ++c) {
                                    wv[c] += W[c][k] * p;
                                    gw[c][0] += W[c][k] * c_ref.dphi[t][qq][k][0];
                                    gw[c][1] += W[c][k] * c_ref.dphi[t][qq][k][1];
                                }
                            }
                            const double wt = c_ref.w[qq] * c_ref.phi[qq][la] * h;
                            for (int k = 0; k < 6; ++k) {
                                const double pk_ = c_ref.phi[qq][k];
                                const double adv = wv[0] * c_ref.dphi[t][qq][k][0] + wv[1] * c_ref.dphi[t][qq][k][1];
                                for (int c = 0; c < 2; ++c) {
                                    for (int d = 0; d < 2; ++d) Nw[c][d][k] += wt * pk_ * gw[c][d];
                                    Nw[c][c][k] += wt * adv;
                                }
                            }
                        }
                    }
                    // read-modify-write of the element's entries in batches: the
                    // entries of one batch are distinct (distinct columns of a
                    // row), so all their loads go out before the first store
                    // (masked entries read the band's first word and write nothing)
                    {
                        int off[24];
                        T old[24];
#pragma unroll
                        for (int k = 0; k < 6; ++k)
#pragma unroll
                            for (int c = 0; c < 2; ++c)
#pragma unroll
                                for (int d = 0; d < 2; ++d) {
                                    const int col = dk[k] + d;
                                    off[4 * k + 2 * c + d] = dk[k] >= 0 ? col * ld + (dv + c - col + S.bw) : 0;
                                }
#pragma unroll
                        for (int i = 0; i < 24; ++i) old[i] = (fv >> (i >> 2)) & 1u ? (T)0 : band[off[i]];
#pragma unroll
                        for (int k = 0; k < 6; ++k) {
                            if (dk[k] < 0) continue;
#pragma unroll
                            for (int c = 0; c < 2; ++c)
#pragma unroll
                                for (int d = 0; d < 2; ++d) {
                                    double v = nue * c_ref.Se[t][c * 6 + la][d * 6 + k] + eta * Nw[c][d][k];
                                    if (c == d) v += edt * h2 * c_ref.Me[t][la][k];
                                    const int i = 4 * k + 2 * c + d;
                                    band[off[i]] = (T)((double)old[i] + v);
                                }
                        }
                    }
                    {
                        int off[6];
                        T old[6];
#pragma unroll
                        for (int v = 0; v < 3; ++v)
#pragma unroll
                            for (int c = 0; c < 2; ++c)
                                off[2 * v + c] = pk[v] >= 0 ? pk[v] * ld + (dv + c - pk[v] + S.bw) : 0;
#pragma unroll
                        for (int i = 0; i < 6; ++i) old[i] = (fp >> (i >> 1)) & 1u ? (T)0 : band[off[i]];
#pragma unroll
                        for (int v = 0; v < 3; ++v)
                            if (pk[v] >= 0)
#pragma unroll
                                for (int c = 0; c < 2; ++c)
                                    band[off[2 * v + c]] = (T)((double)old[2 * v + c] - eta * h * c_ref.Be[t][v][c * 6 + la]);
                    }
                }
            }
            if (dp >= 0) {
                const int lv = p1_local(t, (a >> 1) - ci, (b >> 1) - cj);
                {
                    int off[12];
                    T old[12];
#pragma unroll
                    for (int k = 0; k < 6; ++k)
#pragma unroll
                        for (int d = 0; d < 2; ++d) {
                            const int col = dk[k] + d;
                            off[2 * k + d] = dk[k] >= 0 ? col * ld + (dp - col + S.bw) : 0;
                        }
#pragma unroll
                    for (int i = 0; i < 12; ++i) old[i] = (fv >> (i >> 1)) & 1u ? (T)0 : band[off[i]];
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        if (dk[k] >= 0)
#pragma unroll
                            for (int d = 0; d < 2; ++d)
                                band[off[2 * k + d]] = (T)((double)old[2 * k + d] + eta * h * c_ref.Be[t][lv][d * 6 + k]);
                }
            }
        });
        // Beavers-Joseph term on Gamma edges (x rows, x columns; entries an
        // element has written)
        if (dv >= 0 && S.gamma && 2 * S.y0 + b == 0) {
            const int A0 = 2 * S.x0 + a;
            const int ne = (A0 & 1) ? 1 : 2;
            for (int e = 0; e < ne; ++e) {
                const int ie = (A0 & 1) ? (A0 >> 1) : (A0 >> 1) - 1 + e;
                if (ie < S.x0 || ie >= S.x0 + S.cx) continue;
                const int la = A0 - 2 * ie;
                for (int k = 0; k < 3; ++k) {
                    const int qk = 2 * ie + k - 2 * S.x0;
                    const int dk = A.dof2[S.node_off + qk];
                    if (dk < 0) continue;
                    const double v = eta * cf.beta * h * c_ref.Ge[la][k];
                    put(dv, dk, v);
                }
            }
        }
    }
}

// Oseen residual r = b - K x (FP64) by tiles of RT x RT cells of a box: each
// triangle of the tile (and of a one-cell halo below and to the left) is
// integrated once, for all six of its nodes' rows (the quadrature of the
// convection term shared by them) into LDS; then every node of the tile adds
// the contributions of its triangles in the node-thread order, so a node's
// sum does not depend on the tiling.  Blocks past a box's tile count only
// take part in the norm reduction.  A block takes tiles blockIdx.x,
// blockIdx.x + gridDim.x, ... of its box; with one block per box the norms
// are finished in the block.
constexpr int RT = 8;
constexpr int RT_TRI = 2 * (RT + 1) * (RT + 1);
int residual_tiles(int cx, int cy) { return ((cx + RT - 1) / RT) * ((cy + RT - 1) / RT); }

// Apply mode (b null): r = -K x without norms or flags (part null), systems
// whose conv flag is set skipped.
__global__ __launch_bounds__(256) void k_oseen_residual_tiled(OseenApplyArgs<double> A) {
    const SysDesc S = A.sys[blockIdx.y];
    const Coef &cf = A.co[S.sample];   // the coefficients of the system's sample
    if (A.skip && A.skip[S.sample]) return;
    if (A.conv && A.conv[blockIdx.y]) return;
    const int ntx = (S.cx + RT - 1) / RT, nty = (S.cy + RT - 1) / RT;
    const int ng = 2 * S.N + 1;
    const double h = S.h, h2 = h * h;
    const double eta = cf.eta, edt = cf.eta / cf.dt, nue = cf.nu * cf.eta;
    const double *x = A.x + S.dof_off;
    __shared__ double cv[RT_TRI][6][2];     // velocity rows: (triangle, its node la, component)
    __shared__ double cp[RT_TRI][3];        // pressure rows: (triangle, its vertex)
    const int tid = threadIdx.x;
    double tr[1] = {0.0}, tb[1] = {0.0};                       // the box's norms so far (one block per box)
    const bool act1[1] = {true};
    for (int tile = blockIdx.x; tile < ntx * nty; tile += gridDim.x) {
        double rr = 0.0, bb = 0.0;
        const int tx = tile % ntx, ty = tile / ntx;
        const int ci_lo = tx * RT - 1, cj_lo = ty * RT - 1;    // first (halo) cell of the tile's triangles
        if (tile != (int)blockIdx.x) __syncthreads();          // the previous tile's node pass is done with LDS
        for (int e = tid; e < RT_TRI; e += blockDim.x) {
            const int t = e & 1, cc = e >> 1;
            const int ci = ci_lo + cc % (RT + 1), cj = cj_lo + cc / (RT + 1);
            if (ci < 0 || cj < 0 || ci >= S.cx || cj >= S.cy) continue;
            double W[2][6], X[2][6], Pv[3];
            for (int k = 0; k < 6; ++k) {
                const int qa = 2 * ci + off2a(t, k), qb = 2 * cj + off2b(t, k);
                const long long Gk = (2 * S.x0 + qa) + (long long)ng * (2 * S.y0 + qb);
                const int dk = A.dof2[S.node_off + qa + S.lw2 * qb];
                for (int c = 0; c < 2; ++c) {
                    W[c][k] = A.W1[c][S.zo + Gk];
                    X[c][k] = dk >= 0 ? x[dk + c] : 0.0;
                }
            }
            for (int v = 0; v < 3; ++v) {
                const int pk = A.dof1[S.vert_off + (ci + off1a(t, v)) + S.lw1 * (cj + off1b(t, v))];
                Pv[v] = pk >= 0 ? x[pk] : 0.0;
            }
            // int (N(W) X)_c phi_la for the six test nodes at once
            double Nz[6][2];
            for (int l = 0; l < 6; ++l) Nz[l][0] = Nz[l][1] = 0.0;
            if (cf.convection) {
                for (int q = 0; q < NQ; ++q) {
                    double wv[2] = {0, 0}, gw[2][2] = {{0, 0}, {0, 0}}, zv[2] = {0, 0}, gz[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        const double p = c_ref.phi[q][k];
                        const double dx0 = c_ref.dphi[0][q][k][0], dx1 = c_ref.dphi[1][q][k][0];
                        const double dy0 = c_ref.dphi[0][q][k][1], dy1 = c_ref.dphi[1][q][k][1];
                        const double dx = t ? dx1 : dx0, dy = t ? dy1 : dy0;
                        for (int c = 0; c < 2; ++c) {
                            wv[c] += W[c][k] * p;
                            gw[c][0] += W[c][k] * dx;
                            gw[c][1] += W[c][k] * dy;
                            zv[c] += X[c][k] * p;
                            gz[c][0] += X[c][k] * dx;
                            gz[c][1] += X[c][k] * dy;
                        }
                    }
                    double g[2];
                    for (int c = 0; c < 2; ++c) g[c] = zv[0] * gw[c][0] + zv[1] * gw[c][1] + wv[0] * gz[c][0] + wv[1] * gz[c][1];
#pragma unroll
                    for (int l = 0; l < 6; ++l) {
                        const double wt = c_ref.w[q] * c_ref.phi[q][l];
                        for (int c = 0; c < 2; ++c) Nz[l][c] += wt * g[c];
                    }
                }
                for (int l = 0; l < 6; ++l) { Nz[l][0] *= h; Nz[l][1] *= h; }
            }
            for (int l = 0; l < 6; ++l)
                for (int c = 0; c < 2; ++c) {
                    double m = 0.0, sv = 0.0, bt = 0.0;
                    for (int k = 0; k < 6; ++k) {
                        m += c_ref.Me[t][l][k] * X[c][k];
                        for (int d = 0; d < 2; ++d) sv += c_ref.Se[t][c * 6 + l][d * 6 + k] * X[d][k];
                    }
                    for (int v = 0; v < 3; ++v) bt += c_ref.Be[t][v][c * 6 + l] * Pv[v];
                    cv[e][l][c] = edt * h2 * m + nue * sv + eta * Nz[l][c] - eta * h * bt;
                }
            for (int v = 0; v < 3; ++v) {
                double sv = 0.0;
                for (int d = 0; d < 2; ++d)
                    for (int k = 0; k < 6; ++k) sv += c_ref.Be[t][v][d * 6 + k] * X[d][k];
                cp[e][v] = eta * h * sv;
            }
        }
        __syncthreads();
        // nodes of the tile: lattice columns 2 RT tx .. (the last tile to the box's edge)
        const int a0 = 2 * RT * tx, a1 = tx == ntx - 1 ? 2 * S.cx : 2 * RT * (tx + 1) - 1;
        const int b0 = 2 * RT * ty, b1 = ty == nty - 1 ? 2 * S.cy : 2 * RT * (ty + 1) - 1;
        const int wa = a1 - a0 + 1, cnt = wa * (b1 - b0 + 1);
        for (int idx = tid; idx < cnt; idx += blockDim.x) {
            const int a = a0 + idx % wa, b = b0 + idx / wa;
            const int q = a + S.lw2 * b;
            const int cls = A.cls2[S.node_off + q];
            const bool vertex = !(a & 1) && !(b & 1);
            const int dv = cls == 0 ? A.dof2[S.node_off + q] : -1;
            const int dp = vertex ? A.dof1[S.vert_off + (a >> 1) + S.lw1 * (b >> 1)] : -1;
            if (dv < 0 && dp < 0) continue;
            double yv[2] = {0.0, 0.0}, yq = 0.0;
            for_elements(a, b, S.cx, S.cy, [&](int t, int ci, int cj, int la) {
                const int e = 2 * ((ci - ci_lo) + (RT + 1) * (cj - cj_lo)) + t;
                if (dv >= 0) { yv[0] += cv[e][la][0]; yv[1] += cv[e][la][1]; }
                if (dp >= 0) yq += cp[e][p1_local(t, (a >> 1) - ci, (b >> 1) - cj)];
            });
            // Beavers-Joseph term on Gamma edges (x rows, x columns)
            if (dv >= 0 && S.gamma && 2 * S.y0 + b == 0) {
                const int A0 = 2 * S.x0 + a;
                const int ne = (A0 & 1) ? 1 : 2;
                for (int e2 = 0; e2 < ne; ++e2) {
                    const int ie = (A0 & 1) ? (A0 >> 1) : (A0 >> 1) - 1 + e2;
                    if (ie < S.x0 || ie >= S.x0 + S.cx) continue;
                    const int lg = A0 - 2 * ie;
                    for (int k = 0; k < 3; ++k) {
                        const int dk = A.dof2[S.node_off + (2 * ie + k - 2 * S.x0)];
                        if (dk < 0) continue;
                        yv[0] += eta * cf.beta * h * c_ref.Ge[lg][k] * x[dk];
                    }
                }
            }
            if (dv >= 0)
                for (int c = 0; c < 2; ++c) {
                    const double bv = A.b ? A.b[S.dof_off + dv + c] : 0.0, rv = bv - yv[c];
                    A.r[S.dof_off + dv + c] = rv;
                    rr += rv * rv;
                    bb += bv * bv;
                }
            if (dp >= 0) {
                const double bv = A.b ? A.b[S.dof_off + dp] : 0.0, rv = bv - yq;
                A.r[S.dof_off + dp] = rv;
                rr += rv * rv;
                bb += bv * bv;
            }
        }
        if (A.part) {
            double pr[1] = {rr}, pb[1] = {bb};
            tile_norms(pr, pb, act1, tr, tb, A.part, A.tstride, blockIdx.y, tile);
        }
    }
    if (A.part)
        tile_norms_finish(tr, tb, act1, A.part, A.ticket, A.conv, A.relres, A.sweeps, A.tol, blockIdx.y, A.tstride, ntx * nty);
}

// Local Oseen right-hand sides by the same tiles as the residual: each
// triangle's contributions to its six velocity rows and three pressure rows
// once into LDS, then the node threads (Dirichlet values, sources, Gamma
// terms) add their triangles in the node-thread order.
__global__ __launch_bounds__(256) void k_oseen_rhs_tiled(OseenArgs A) {
    const SysDesc S = A.sys[blockIdx.y];
    const Coef &cf = A.co[S.sample];   // the coefficients of the system's sample
    if (A.skip && A.skip[S.sample]) return;
    const int ntx = (S.cx + RT - 1) / RT, nty = (S.cy + RT - 1) / RT;
    if ((int)blockIdx.x >= ntx * nty) return;
    const int tx = (int)blockIdx.x % ntx, ty = (int)blockIdx.x / ntx;
    const int ci_lo = tx * RT - 1, cj_lo = ty * RT - 1;
    const int nloc = S.lw2 * S.lh2;
    const int ng = 2 * S.N + 1, ng1 = S.N + 1;
    const double h = S.h, h2 = h * h;
    const double eta = cf.eta, edt = cf.eta / cf.dt, nue = cf.nu * cf.eta;
    __shared__ double cv[RT_TRI][6][2];
    __shared__ double cp[RT_TRI][3];
    const int tid = threadIdx.x;
    if (A.ir.conv && blockIdx.x == 0 && tid == 0) {
        A.ir.conv[blockIdx.y] = 0;
        A.ir.relres[blockIdx.y] = 0.0;
        A.ir.sweeps[blockIdx.y] = 0;
    }
    for (int e = tid; e < RT_TRI; e += blockDim.x) {
        const int t = e & 1, cc = e >> 1;
        const int ci = ci_lo + cc % (RT + 1), cj = cj_lo + cc / (RT + 1);
        if (ci < 0 || cj < 0 || ci >= S.cx || cj >= S.cy) continue;
        double W[2][6], Z[2][6], Y[2][6], O[2][6], P[3];
        for (int k = 0; k < 6; ++k) {
            const int qa = 2 * ci + off2a(t, k), qb = 2 * cj + off2b(t, k);
            const int qk = qa + S.lw2 * qb;
            const long long Gk = (2 * S.x0 + qa) + (long long)ng * (2 * S.y0 + qb);
            for (int c = 0; c < 2; ++c) {
                W[c][k] = A.W1[c][S.zo + Gk];
                Z[c][k] = oseen_z(S, A, c, qk, Gk);
                Y[c][k] = W[c][k] + Z[c][k];
                O[c][k] = (A.W0[c] ? A.W0[c][S.zo + Gk] : 0.0) + (A.e_old ? A.e_old[S.e2_off + (long long)c * nloc + qk] : 0.0)
                          - W[c][k] - Z[c][k];
            }
        }
        for (int k = 0; k < 3; ++k)
            P[k] = A.Pp[S.zo + (S.x0 + ci + off1a(t, k)) + (long long)ng1 * (S.y0 + cj + off1b(t, k))];
        // int ((W.grad)W + N(W) Z)_c phi_la for the six test nodes at once
        double CN[6][2];
        for (int l = 0; l < 6; ++l) CN[l][0] = CN[l][1] = 0.0;
        if (cf.convection) {
            for (int q = 0; q < NQ; ++q) {
                double wv[2] = {0, 0}, gw[2][2] = {{0, 0}, {0, 0}}, zv[2] = {0, 0}, gz[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const double p = c_ref.phi[q][k];
                    const double dx0 = c_ref.dphi[0][q][k][0], dx1 = c_ref.dphi[1][q][k][0];
                    const double dy0 = c_ref.dphi[0][q][k][1], dy1 = c_ref.dphi[1][q][k][1];
                    const double dx = t ? dx1 : dx0, dy = t ? dy1 : dy0;
                    for (int c = 0; c < 2; ++c) {
                        wv[c] += W[c][k] * p;
                        gw[c][0] += W[c][k] * dx;
                        gw[c][1] += W[c][k] * dy;
                        zv[c] += Z[c][k] * p;
                        gz[c][0] += Z[c][k] * dx;
                        gz[c][1] += Z[c][k] * dy;
                    }
                }
                double g[2];
                for (int c = 0; c < 2; ++c)
                    g[c] = wv[0] * gw[c][0] + wv[1] * gw[c][1] + (zv[0] * gw[c][0] + zv[1] * gw[c][1] + wv[0] * gz[c][0] + wv[1] * gz[c][1]);
#pragma unroll
                for (int l = 0; l < 6; ++l) {
                    const double wt = c_ref.w[q] * c_ref.phi[q][l];
                    for (int c = 0; c < 2; ++c) CN[l][c] += wt * g[c];
                }
            }
            for (int l = 0; l < 6; ++l) { CN[l][0] *= h; CN[l][1] *= h; }
        }
        for (int l = 0; l < 6; ++l)
            for (int c = 0; c < 2; ++c) {
                double m = 0.0, sv = 0.0, bt = 0.0;
                for (int k = 0; k < 6; ++k) {
                    m += c_ref.Me[t][l][k] * O[c][k];
                    for (int d = 0; d < 2; ++d) sv += c_ref.Se[t][c * 6 + l][d * 6 + k] * Y[d][k];
                }
                for (int v = 0; v < 3; ++v) bt += c_ref.Be[t][v][c * 6 + l] * P[v];
                cv[e][l][c] = edt * h2 * m - nue * sv - eta * CN[l][c] + eta * h * bt;
            }
        for (int v = 0; v < 3; ++v) {
            double sv = 0.0;
            for (int d = 0; d < 2; ++d)
                for (int k = 0; k < 6; ++k) sv += c_ref.Be[t][v][d * 6 + k] * Y[d][k];
            cp[e][v] = -eta * h * sv;
        }
    }
    __syncthreads();
    const int a0 = 2 * RT * tx, a1 = tx == ntx - 1 ? 2 * S.cx : 2 * RT * (tx + 1) - 1;
    const int b0 = 2 * RT * ty, b1 = ty == nty - 1 ? 2 * S.cy : 2 * RT * (ty + 1) - 1;
    const int wa = a1 - a0 + 1, cnt = wa * (b1 - b0 + 1);
    double *en = A.e_new + S.e2_off;
    for (int idx = tid; idx < cnt; idx += blockDim.x) {
        const int a = a0 + idx % wa, b = b0 + idx / wa;
        const int q = a + S.lw2 * b;
        const long long G = (2 * S.x0 + a) + (long long)ng * (2 * S.y0 + b);
        const int cls = A.cls2[S.node_off + q];
        const bool vertex = !(a & 1) && !(b & 1);
        const int vq = vertex ? (a >> 1) + S.lw1 * (b >> 1) : -1;
        const bool prow = vertex && A.cls1[S.vert_off + vq] == 0;
        if (cls != 0)
            for (int c = 0; c < 2; ++c) en[(long long)c * nloc + q] = oseen_z(S, A, c, q, G);
        if (vertex && !prow) A.e_new1[S.e1_off + vq] = 0.0;
        if (cls != 0 && !prow) continue;
        double rv[2] = {0.0, 0.0}, rq = 0.0;
        if (cls == 0)
            for (int c = 0; c < 2; ++c)
                rv[c] = eta * (A.load[c][0][S.zo + G] * A.tf[0] + A.load[c][1][S.zo + G] * A.tf[1] + A.load[c][2][S.zo + G] * A.tf[2]);
        for_elements(a, b, S.cx, S.cy, [&](int t, int ci, int cj, int la) {
            const int e = 2 * ((ci - ci_lo) + (RT + 1) * (cj - cj_lo)) + t;
            if (cls == 0) { rv[0] += cv[e][la][0]; rv[1] += cv[e][la][1]; }
            if (prow) rq += cp[e][p1_local(t, (a >> 1) - ci, (b >> 1) - cj)];
        });
        // Gamma edges (conduit bottom row): Beavers-Joseph on the x rows and the
        // lagged p_F^n terms -(eta/rho) int p_F v.n_c - c_tau int d_x p_F v_x
        if (cls == 0 && S.gamma && 2 * S.y0 + b == 0) {
            const int A0 = 2 * S.x0 + a;
            const int ne = (A0 & 1) ? 1 : 2;
            for (int e2 = 0; e2 < ne; ++e2) {
                const int ie = (A0 & 1) ? (A0 >> 1) : (A0 >> 1) - 1 + e2;
                if (ie < S.x0 || ie >= S.x0 + S.cx) continue;
                const int lg = A0 - 2 * ie;
                double bj = 0.0, pg = 0.0, pgx = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const int qk = (2 * ie + k - 2 * S.x0);     // box-local, row 0
                    const long long Gk = 2 * ie + k;           // grid conduit row 0
                    bj += c_ref.Ge[lg][k] * (A.W1[0][S.zo + Gk] + oseen_z(S, A, 0, qk, Gk));
                    const double pf = A.PF0[S.zo + (2 * ie + k) + (long long)ng * (2 * S.N)];   // porous top row
                    pg += c_ref.Ge[lg][k] * pf;
                    pgx += c_ref.Gxe[lg][k] * pf;
                }
                rv[0] -= eta * cf.beta * h * bj + cf.ctau * pgx;
                rv[1] += eta / cf.rho * h * pg;
            }
        }
        auto put = [&](long long row, double v) {
            A.b[row] = v;
            if (A.ir.r) { A.ir.r[row] = v; A.ir.x[row] = 0.0; }
        };
        if (cls == 0) {
            const long long d = S.dof_off + A.dof2[S.node_off + q];
            put(d, rv[0]);
            put(d + 1, rv[1]);
        }
        if (prow) put(S.dof_off + A.dof1[S.vert_off + vq], rq);
    }
}

// Porous residuals of the three fields by the same tiles of cells: each
// triangle's contributions to its six rows once into LDS, the node threads
// add their triangles in the node-thread order.  A converged field is left
// alone; blocks past a box's tile count only take part in the reductions.
__global__ __launch_bounds__(256) void k_porous_residual_tiled(ResidualArgs R) {
    const SysDesc S = R.sys[blockIdx.y];
    const Coef &cf = R.co[S.sample];   // the coefficients of the system's sample
    if (R.skip && R.skip[S.sample]) return;
    const int id0 = blockIdx.y * 3;
    bool act[3];
    for (int f = 0; f < 3; ++f) act[f] = !R.conv[id0 + f];
    if (!act[0] && !act[1] && !act[2]) return;
    const int ntx = (S.cx + RT - 1) / RT, nty = (S.cy + RT - 1) / RT;
    const double h2 = S.h * S.h;
    double cm[3], ck[3];
    for (int f = 0; f < 3; ++f) { cm[f] = (cf.tau[f] + porous_x(cf, f)) * h2; ck[f] = cf.kap[f]; }
    const double *x = R.x + S.dof_off, *b = R.b + S.dof_off;
    double *r = R.r + S.dof_off;
    const long long nd = S.ndof;
    __shared__ double cy[RT_TRI][6][3];     // (triangle, its node la, field)
    const int tid = threadIdx.x;
    double tr[3] = {0.0, 0.0, 0.0}, tb[3] = {0.0, 0.0, 0.0};   // the box's norms so far (one block per box)
    for (int tile = blockIdx.x; tile < ntx * nty; tile += gridDim.x) {
        double rr[3] = {0.0, 0.0, 0.0}, bb[3] = {0.0, 0.0, 0.0};
        const int tx = tile % ntx, ty = tile / ntx;
        const int ci_lo = tx * RT - 1, cj_lo = ty * RT - 1;
        if (tile != (int)blockIdx.x) __syncthreads();          // the previous tile's node pass is done with LDS
        for (int e = tid; e < RT_TRI; e += blockDim.x) {
            const int t = e & 1, cc = e >> 1;
            const int ci = ci_lo + cc % (RT + 1), cj = cj_lo + cc / (RT + 1);
            if (ci < 0 || cj < 0 || ci >= S.cx || cj >= S.cy) continue;
            double X[3][6];
            for (int k = 0; k < 6; ++k) {
                const int dk = R.dof2[S.node_off + (2 * ci + off2a(t, k)) + S.lw2 * (2 * cj + off2b(t, k))];
                for (int f = 0; f < 3; ++f) X[f][k] = dk >= 0 && act[f] ? x[f * nd + dk] : 0.0;
            }
            for (int l = 0; l < 6; ++l) {
                double y[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < 6; ++k) {
                    const double me = c_ref.Me[t][l][k], ke = c_ref.Ke[t][l][k];
                    for (int f = 0; f < 3; ++f) y[f] += (cm[f] * me + ck[f] * ke) * X[f][k];
                }
                for (int f = 0; f < 3; ++f) cy[e][l][f] = y[f];
            }
        }
        __syncthreads();
        const int a0 = 2 * RT * tx, a1 = tx == ntx - 1 ? 2 * S.cx : 2 * RT * (tx + 1) - 1;
        const int b0 = 2 * RT * ty, b1 = ty == nty - 1 ? 2 * S.cy : 2 * RT * (ty + 1) - 1;
        const int wa = a1 - a0 + 1, cnt = wa * (b1 - b0 + 1);
        for (int idx = tid; idx < cnt; idx += blockDim.x) {
            const int a = a0 + idx % wa, bq = b0 + idx / wa;
            const int dq = R.dof2[S.node_off + a + S.lw2 * bq];
            if (dq < 0) continue;
            double y[3] = {0.0, 0.0, 0.0};
            for_elements(a, bq, S.cx, S.cy, [&](int t, int ci, int cj, int la) {
                const int e = 2 * ((ci - ci_lo) + (RT + 1) * (cj - cj_lo)) + t;
                for (int f = 0; f < 3; ++f) y[f] += cy[e][la][f];
            });
            for (int f = 0; f < 3; ++f) {
                if (!act[f]) continue;
                const double bv = b[f * nd + dq], rv = bv - y[f];
                r[f * nd + dq] = rv;
                rr[f] += rv * rv;
                bb[f] += bv * bv;
            }
        }
        tile_norms(rr, bb, act, tr, tb, R.part, R.tstride, id0, tile);
    }
    tile_norms_finish(tr, tb, act, R.part, R.ticket, R.conv, R.relres, R.sweeps, R.tol, id0, R.tstride, ntx * nty);
}

// Local porous right-hand sides by the same tiles: each triangle's mass and
// stiffness contributions to its six rows (three fields) once into LDS, then
// the node threads (Dirichlet values, sources, the Gamma term) add their
// triangles in the node-thread order.
__global__ __launch_bounds__(256) void k_porous_rhs_tiled(PorousArgs A) {
    const SysDesc S = A.sys[blockIdx.y];
    const Coef &cf = A.co[S.sample];   // the coefficients of the system's sample
    const int ntx = (S.cx + RT - 1) / RT, nty = (S.cy + RT - 1) / RT;
    if ((int)blockIdx.x >= ntx * nty) return;
    const int tx = (int)blockIdx.x % ntx, ty = (int)blockIdx.x / ntx;
    const int ci_lo = tx * RT - 1, cj_lo = ty * RT - 1;
    const int nloc = S.lw2 * S.lh2;
    const int ng = 2 * S.N + 1;
    const double h = S.h, h2 = h * h;
    __shared__ double cr[RT_TRI][6][3];     // (triangle, its node la, field)
    const int tid = threadIdx.x;
    if (A.ir.conv && blockIdx.x == 0 && tid < 3) {
        A.ir.conv[3 * blockIdx.y + tid] = 0;
        A.ir.relres[3 * blockIdx.y + tid] = 0.0;
        A.ir.sweeps[3 * blockIdx.y + tid] = 0;
    }
    for (int e = tid; e < RT_TRI; e += blockDim.x) {
        const int t = e & 1, cc = e >> 1;
        const int ci = ci_lo + cc % (RT + 1), cj = cj_lo + cc / (RT + 1);
        if (ci < 0 || cj < 0 || ci >= S.cx || cj >= S.cy) continue;
        double M3[3][6], X3[3][6];      // mass-term and stiffness-term nodal values per field
        for (int k = 0; k < 6; ++k) {
            const int qa = 2 * ci + off2a(t, k), qb = 2 * cj + off2b(t, k);
            const int qk = qa + S.lw2 * qb;
            const long long Gk = (2 * S.x0 + qa) + (long long)ng * (2 * S.y0 + qb);
            const bool dir = A.cls2[S.node_off + qk] == 1;
            double O[3], X[3];
            for (int g = 0; g < 3; ++g) {
                const double p1 = A.P1[g] ? A.P1[g][S.zo + Gk] : 0.0;
                O[g] = (A.P0[g] ? A.P0[g][S.zo + Gk] : 0.0) + A.e_old[S.e2_off + (long long)g * nloc + qk];
                X[g] = p1 + (dir ? A.ex[g][Gk] * A.tf[0] - p1 : 0.0);
            }
            for (int f = 0; f < 3; ++f) {
                double m = cf.tau[f] * (O[f] - X[f]) - porous_x(cf, f) * X[f];
                if (f == 0) m += cf.sst * O[1];
                if (f == 1) m += cf.s * O[2] + cf.sst * O[0];
                if (f == 2) m += cf.s * O[1];
                M3[f][k] = m;
                X3[f][k] = X[f];
            }
        }
        for (int l = 0; l < 6; ++l) {
            double mv[3] = {0.0, 0.0, 0.0}, kv[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < 6; ++k) {
                const double me = c_ref.Me[t][l][k], ke = c_ref.Ke[t][l][k];
                for (int f = 0; f < 3; ++f) { mv[f] += me * M3[f][k]; kv[f] += ke * X3[f][k]; }
            }
            for (int f = 0; f < 3; ++f) cr[e][l][f] = h2 * mv[f] - cf.kap[f] * kv[f];
        }
    }
    __syncthreads();
    const int a0 = 2 * RT * tx, a1 = tx == ntx - 1 ? 2 * S.cx : 2 * RT * (tx + 1) - 1;
    const int b0 = 2 * RT * ty, b1 = ty == nty - 1 ? 2 * S.cy : 2 * RT * (ty + 1) - 1;
    const int wa = a1 - a0 + 1, cnt = wa * (b1 - b0 + 1);
    for (int idx = tid; idx < cnt; idx += blockDim.x) {
        const int a = a0 + idx % wa, b = b0 + idx / wa;
        const int q = a + S.lw2 * b;
        const long long G = (2 * S.x0 + a) + (long long)ng * (2 * S.y0 + b);
        const int cls = A.cls2[S.node_off + q];
        if (cls != 0) {
            for (int f = 0; f < 3; ++f) A.e_new[S.e2_off + (long long)f * nloc + q] = porous_z(S, A, f, q, G);
            continue;
        }
        // sources at t_{n+1}
        double r[3];
        for (int f = 0; f < 3; ++f) r[f] = A.load[f][0][S.zo + G] * A.tf[0] + A.load[f][1][S.zo + G] * A.tf[1];
        for_elements(a, b, S.cx, S.cy, [&](int t, int ci, int cj, int la) {
            const int e = 2 * ((ci - ci_lo) + (RT + 1) * (cj - cj_lo)) + t;
            for (int f = 0; f < 3; ++f) r[f] += cr[e][la][f];
        });
        // + <u^n . n_c, v_F>_Gamma = -int_Gamma v_F u_y^n on the porous top row
        if (S.gamma && 2 * S.y0 + b == 2 * S.N && A.Uy0) {
            const int A0 = 2 * S.x0 + a;
            const int ne = (A0 & 1) ? 1 : 2;
            for (int e2 = 0; e2 < ne; ++e2) {
                const int ie = (A0 & 1) ? (A0 >> 1) : (A0 >> 1) - 1 + e2;
                if (ie < S.x0 || ie >= S.x0 + S.cx) continue;
                const int lg = A0 - 2 * ie;
                double sg = 0.0;
                for (int k = 0; k < 3; ++k) sg += c_ref.Ge[lg][k] * A.Uy0[S.zo + 2 * ie + k];   // conduit Gamma row b = 0
                r[0] -= h * sg;
            }
        }
        const int d = A.dof2[S.node_off + q];
        for (int f = 0; f < 3; ++f) {
            const long long row = S.dof_off + (long long)f * S.ndof + d;
            A.b[row] = r[f];
            if (A.ir.r) { A.ir.r[row] = r[f]; A.ir.x[row] = 0.0; }
        }
    }
}

// Jacobian rows of a few large-lattice Oseen systems (the coarse Navier-Stokes
// Jacobian: one system of a few hundred nodes, where one thread per node leaves
// the GPU idle).  One wavefront per lattice node: lane 8 e + s takes triangle
// slot e of the node (the visiting order of for_elements) and column node s of
// that triangle, so the quadrature of all triangles runs at once.  The node's
// rows are summed in LDS, triangle after triangle in that same order (the
// entries of one triangle are distinct columns), and then stored whole: every
// band entry of a row is written, untouched ones as zero, so the band needs no
// clearing.  Same entries, same summation order per entry as the node-thread
// kernel's assembly mode.
template <typename T>
__global__ __launch_bounds__(64) void k_oseen_rows(OseenApplyArgs<T> A) {
    const SysDesc S = A.sys[blockIdx.y];
    const Coef &cf = A.co[S.sample];   // the coefficients of the system's sample
    if (A.skip && A.skip[S.sample]) return;
    const int q = blockIdx.x;
    const int nloc = S.lw2 * S.lh2;
    if (q >= nloc) return;
    const int lane = threadIdx.x;
    const int a = q % S.lw2, b = q / S.lw2;
    const int cls = A.cls2[S.node_off + q];
    const bool vertex = !(a & 1) && !(b & 1);
    const int dv = cls == 0 ? A.dof2[S.node_off + q] : -1;
    const int dp = vertex ? A.dof1[S.vert_off + (a >> 1) + S.lw1 * (b >> 1)] : -1;
    if (dv < 0 && dp < 0) return;
    const int ng = 2 * S.N + 1, ld = 2 * S.bw + 1;
    const double h = S.h, h2 = h * h;
    const double eta = cf.eta, edt = cf.eta / cf.dt, nue = cf.nu * cf.eta;
    extern __shared__ double rows_dyn[];
    T *row = reinterpret_cast<T *>(rows_dyn);            // [3][ld]: rows dv, dv + 1, dp
    for (int j = lane; j < 3 * ld; j += 64) row[j] = (T)0;
    // this lane's triangle and column node
    const int e = lane >> 3, s = lane & 7;
    const int t = e & 1;
    const int ci0 = (a - 1) >> 1 < 0 ? 0 : ((a - 1) >> 1);
    const int ci1 = (a >> 1) < S.cx ? (a >> 1) : S.cx - 1;
    const int cj0 = (b - 1) >> 1 < 0 ? 0 : ((b - 1) >> 1);
    const int cj1 = (b >> 1) < S.cy ? (b >> 1) : S.cy - 1;
    const int ci = ci0 + ((e >> 1) & 1), cj = cj0 + (e >> 2);
    const int la_ = a - 2 * ci, lb_ = b - 2 * cj;
    bool on = ci <= ci1 && cj <= cj1 && la_ >= 0 && la_ <= 2 && lb_ >= 0 && lb_ <= 2;
    const int la = on ? p2_local(t, la_, lb_) : -1;
    on = on && la >= 0 && s < 6;
    // entry values and their row slots / columns
    double vv[2][2] = {{0, 0}, {0, 0}}, vp[2] = {0, 0}, vq[2] = {0, 0};
    int dks = -1, pks = -1;
    if (on) {
        const int k = s;
        dks = A.dof2[S.node_off + (2 * ci + off2a(t, k)) + S.lw2 * (2 * cj + off2b(t, k))];
        if (k < 3) pks = A.dof1[S.vert_off + (ci + off1a(t, k)) + S.lw1 * (cj + off1b(t, k))];
        if (dv >= 0) {
            double Nw[2][2] = {{0, 0}, {0, 0}};
            if (cf.convection) {
                double W[2][6];
                for (int kk = 0; kk < 6; ++kk) {
                    const long long Gk = (2 * S.x0 + 2 * ci + off2a(t, kk)) + (long long)ng * (2 * S.y0 + 2 * cj + off2b(t, kk));
                    for (int c = 0; c < 2; ++c) W[c][kk] = A.W1[c][S.zo + Gk];
                }
                for (int qq = 0; qq < NQ; ++qq) {
                    double wv[2] = {0, 0}, gw[2][2] = {{0, 0}, {0, 0}};
                    for (int kk = 0; kk < 6; ++kk) {
                        const double p = c_ref.phi[qq][kk];
                        for (int c = 0; c < 2; ++c) {
                            wv[c] += W[c][kk] * p;
                            gw[c][0] += W[c][kk] * c_ref.dphi[t][qq][kk][0];
                            gw[c][1] += W[c][kk] * c_ref.dphi[t][qq][kk][1];
                        }
                    }
                    const double wt = c_ref.w[qq] * c_ref.phi[qq][la] * h;
                    const double pk_ = c_ref.phi[qq][k];
                    const double adv = wv[0] * c_ref.dphi[t][qq][k][0] + wv[1] * c_ref.dphi[t][qq][k][1];
                    for (int c = 0; c < 2; ++c) {
                        for (int d = 0; d < 2; ++d) Nw[c][d] += wt * pk_ * gw[c][d];
                        Nw[c][c] += wt * adv;
                    }
                }
            }
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d) {
                    double v = nue * c_ref.Se[t][c * 6 + la][d * 6 + k] + eta * Nw[c][d];
                    if (c == d) v += edt * h2 * c_ref.Me[t][la][k];
                    vv[c][d] = v;
                }
            if (k < 3)
                for (int c = 0; c < 2; ++c) vp[c] = eta * h * c_ref.Be[t][k][c * 6 + la];
        }
        if (dp >= 0) {
            const int lv = p1_local(t, (a >> 1) - ci, (b >> 1) - cj);
            for (int d = 0; d < 2; ++d) vq[d] = eta * h * c_ref.Be[t][lv][d * 6 + k];
        }
    }
    // triangle after triangle: lanes of one triangle touch distinct columns,
    // and the LDS operations of one wavefront complete in program order
    auto add = [&](int r, int col, int rowi, double v) {
        T &x = row[r * ld + (col - rowi + S.bw)];
        x = (T)((double)x + v);
    };
    for (int ee = 0; ee < 8; ++ee) {
        if (on && e == ee) {
            if (dv >= 0 && dks >= 0)
                for (int c = 0; c < 2; ++c)
                    for (int d = 0; d < 2; ++d) add(c, dks + d, dv + c, vv[c][d]);
            if (dv >= 0 && pks >= 0)
                for (int c = 0; c < 2; ++c) {
                    T &x = row[c * ld + (pks - (dv + c) + S.bw)];
                    x = (T)((double)x - vp[c]);
                }
            if (dp >= 0 && dks >= 0)
                for (int d = 0; d < 2; ++d) add(2, dks + d, dp, vq[d]);
        }
        __builtin_amdgcn_wave_barrier();
    }
    // Beavers-Joseph term on Gamma edges (x rows, x columns), after the triangles
    if (lane == 0 && dv >= 0 && S.gamma && 2 * S.y0 + b == 0) {
        const int A0 = 2 * S.x0 + a;
        const int ne = (A0 & 1) ? 1 : 2;
        for (int e2 = 0; e2 < ne; ++e2) {
            const int ie = (A0 & 1) ? (A0 >> 1) : (A0 >> 1) - 1 + e2;
            if (ie < S.x0 || ie >= S.x0 + S.cx) continue;
            const int lg = A0 - 2 * ie;
            for (int k = 0; k < 3; ++k) {
                const int dk = A.dof2[S.node_off + 2 * ie + k - 2 * S.x0];
                if (dk < 0) continue;
                add(0, dk, dv, eta * cf.beta * h * c_ref.Ge[lg][k]);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    // whole rows into the column-major band: entry (r, col) at col * ld + r - col + bw
    T *band = A.band + S.band_off;
    for (int r = 0; r < 3; ++r) {
        const int R = r < 2 ? (dv >= 0 ? dv + r : -1) : dp;
        if (R < 0) continue;
        for (int j = lane; j < ld; j += 64) {
            const int col = R - S.bw + j;
            if (col >= 0 && col < S.ndof) band[(long long)col * ld + (2 * S.bw - j)] = row[r * ld + j];
        }
    }
}

__device__ __forceinline__ void oseen_finalize_rows(const FinalizeArgs &F, const SysDesc &S, int start, int stride) {
    const int nloc = S.lw2 * S.lh2, nv = S.lw1 * S.lh1;
    for (int q = start; q < nloc; q += stride) {
        const int d = F.dof2[S.node_off + q];
        if (d < 0) continue;
        F.e_new[S.e2_off + q] = F.x[S.dof_off + d];
        F.e_new[S.e2_off + nloc + q] = F.x[S.dof_off + d + 1];
    }
    for (int v = start; v < nv; v += stride) {
        const int d = F.dof1[S.vert_off + v];
        if (d >= 0) F.e_new1[S.e1_off + v] = F.x[S.dof_off + d];
    }
}
__global__ __launch_bounds__(GB) void k_oseen_finalize(FinalizeArgs F) {
    const SysDesc S = F.sys[blockIdx.y];
    if (F.skip && F.skip[S.sample]) return;
    record_ir_totals(F.acc);
    oseen_finalize_rows(F, S, blockIdx.x * GB + threadIdx.x, gridDim.x * GB);
}

// ---------------------------------------------------------------------------
// Pivot and growth monitor of one band factorisation.  Each thread keeps the
// largest magnitude it has seen of a matrix entry (amax), of an entry of U
// (umax) and of a pivot reciprocal (dmax); the workgroup reduces them once at
// the end of the kernel.  The smallest pivot relative to the largest entry is
// 1 / (dmax amax) and the growth factor umax / amax; the thresholds of
// lu_tiny and lu_growth_limit raise flag bit 2, and both values go to the
// run-long maxima of B.stat.
struct LuMon {
    float amax = 0.f, umax = 0.f, dmax = 0.f;
    template <typename T> __device__ __forceinline__ void a(T v) { amax = fmaxf(amax, (float)fabs(v)); }
    template <typename T> __device__ __forceinline__ void u(T v) { umax = fmaxf(umax, (float)fabs(v)); }
    template <typename T> __device__ __forceinline__ void d(T v) { dmax = fmaxf(dmax, (float)fabs(v)); }
};
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
// every thread of the workgroup calls this once, after its last barrier
template <typename T, int NWAVES>
__device__ void lu_monitor_finish(const LuMon &m, const BandArgs<T> &B) {
    __shared__ float red[3][NWAVES];
    const float a = wave_max(m.amax), u = wave_max(m.umax), d = wave_max(m.dmax);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][wv] = a; red[1][wv] = u; red[2][wv] = d; }
    __syncthreads();
    if (threadIdx.x == 0) {
        float A = 0.f, U = 0.f, D = 0.f;
        for (int w = 0; w < NWAVES; ++w) { A = fmaxf(A, red[0][w]); U = fmaxf(U, red[1][w]); D = fmaxf(D, red[2][w]); }
        if (A > 0.f) {
            const float growth = U / A, invpiv = D * A;      // invpiv: max|a| / min|u_kk|
            const bool bad = !(invpiv * lu_tiny<T>() < 1.f) || !(growth <= lu_growth_limit<T>());
            if (bad) atomicOr(B.flags, 4);
            if (B.stat) {
                // non-negative floats order like their bit patterns
                atomicMax(reinterpret_cast<unsigned *>(B.stat), __float_as_uint(isfinite(growth) ? growth : INFINITY));
                atomicMax(reinterpret_cast<unsigned *>(B.stat) + 1, __float_as_uint(isfinite(invpiv) ? invpiv : INFINITY));
            }
        }
    }
}

// Band LU without pivoting.  One workgroup per system; the active window of
// WR x WC entries (rows k..k+WR-1, columns k..k+WC-1 relative to the current
// pivot k) lives in registers, thread (tr, tc) holding an RB x CB block.
// Each step shifts the window by one along the diagonal while applying the
// rank-one update; block boundary rows/columns travel through LDS.  Factors
// overwrite the column-major band (entry (i,j) at j*(2bw+1) + i - j + bw).
// Requires WR, WC > bw.
//
// Memory traffic is kept off the critical path: every thread issues the same
// number of global loads and stores per step (out-of-range lanes load a valid
// address and discard it, or store into a private dummy slot), so the
// compiler can wait on exactly the load issued D steps earlier instead of
// draining the memory queue; barriers only order LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The W x W window (W = TP*RB) never moves.  Row
// slot rho holds the one window row congruent to rho mod W (owned by thread
// row rho / RB, register rho % RB), column slots likewise.  At step k the
// pivot row slot k mod W is output as U(k, .) and refilled with the entering
// row k+W; the pivot column slot becomes L(., k) and is refilled with column
// k+W.  Unrolling the step loop by RB steps makes the pivot register index
// static, so only the pivot row and column (2W values) cross LDS per step;
// entering values are prefetched RB steps ahead.  Requires W > bw.
template <typename T, int TP, int RB>
__global__ __launch_bounds__(TP *TP) void k_band_lu(BandArgs<T> B) {
    constexpr int NT = TP * TP, W = TP * RB, U = RB, NE = 2 * W, NI = (NE + NT - 1) / NT;
    const BandSys Sy = B.sys[blockIdx.x];
    if (B.skip && B.skip[blockIdx.x]) return;
    const int n = Sy.n, bw = Sy.bw, ld = 2 * bw + 1;
    const T *M = B.band + Sy.off;
    // factors in the solves' layout (fac_pos): R = ldf slots per column,
    // L by columns, U row-scaled by columns in reverse order, 1 / U(k, k)
    const int ldf = Sy.ldf, nrf = ldf >> 6, R = ldf;
    T *Lr = B.fac + Sy.foff, *Ur = Lr + (long long)n * ldf, *Di = Ur + (long long)n * ldf;
    T *dummy = B.dummy + ((long long)blockIdx.x * NT + threadIdx.x) * NI;
    __shared__ T ubuf[2][W];       // pivot row by column slot
    __shared__ T lbuf[2][W];       // pivot column by row slot
    __shared__ T ent[2][NE];       // entering row by column slot, then entering column by row slot
    const int tid = threadIdx.x, tr = tid / TP, tc = tid % TP;
    LuMon mon;
    T a[RB][RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int jj = 0; jj < RB; ++jj) {
            const long long gi = tr * RB + i, gj = tc * RB + jj, d = gi - gj;
            const bool ok = gi < n && gj < n && d <= bw && d >= -bw;
            const T v = M[ok ? gj * ld + d + bw : 0];
            a[i][jj] = ok ? v : T(0);
            mon.a(a[i][jj]);
        }
    // Per-thread items q = tid + it*NT (q < 2W).  Fetch (for step kk): q < W is
    // A(kk+W, kk+1+q), W <= q is A(kk+1+e, kk+W) with e = q - W; both at a fixed
    // offset plus kk*ld, valid while kk < fend.  Output (step k): q < W is
    // L(k+q, k) (q >= 1) from lbuf, W <= q is U(k, k+c) (c = q - W) from ubuf;
    // stores below a per-item bound, rotated slot tracked incrementally.
    int foff[NI], fend[NI], soff[NI], send[NI], qq[NI], srot[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int q = tid + it * NT;
        qq[it] = q < NE ? q : 0;
        if (q < W) {
            const int d = W - 1 - q;
            foff[it] = (1 + q) * ld + d + bw;
            fend[it] = (d <= bw) ? min(n - W, n - 1 - q) : 0;
            soff[it] = 0;                              // Lr + k*ldf + fac_pos(srot), srot = (k + q) mod R
            srot[it] = q % R;
            send[it] = (q >= 1 && q <= bw) ? n - q : 0;
        } else if (q < NE) {
            const int e = q - W, d = 1 + e - W;
            foff[it] = W * ld + d + bw;
            fend[it] = (d >= -bw) ? min(n - 1 - e, n - W) : 0;
            soff[it] = -e * ldf;                       // Ur + (n-1-k-e)*ldf + fac_pos((n-1-k) mod R); e = 0 -> Di[k]
            srot[it] = 0;
            send[it] = e <= bw ? n - e : 0;
        } else {
            foff[it] = soff[it] = srot[it] = 0;
            fend[it] = send[it] = 0;
        }
    }
    T fifo[U][NI];
#pragma unroll
    for (int s = 0; s < U; ++s)
#pragma unroll
        for (int it = 0; it < NI; ++it) {
            fifo[s][it] = *(s < fend[it] ? M + (foff[it] + s * ld) : B.zero);
            mon.a(fifo[s][it]);
        }
    int bad = 0;
    int kw = 0;                                     // k0 mod W (a multiple of U)
    int rk = (n - 1) % R;                           // (n-1-k) mod R
    for (int k0 = 0; k0 < n; k0 += U) {
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const int k = k0 + s;
            if (k >= n) break;
            const int ps = s;                       // pivot register index (static)
            const int kmod = kw + s;                // k mod W
            const int ow = kmod / RB;               // owner thread row / column of the pivot slots
            const bool orow = tr == ow, ocol = tc == ow;
            const int buf = k & 1;
            if (orow) {
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) ubuf[buf][tc * RB + jj] = a[ps][jj];
            }
            if (ocol) {
#pragma unroll
                for (int i = 0; i < RB; ++i) lbuf[buf][tr * RB + i] = a[i][ps];
            }
            // entering values of this step (fetched U steps ago) to their slots
#pragma unroll
            for (int it = 0; it < NI; ++it) {
                const int q = tid + it * NT;
                if (q < NE) {
                    const int base = q < W ? 0 : W, o = q < W ? q : q - W;
                    int sl = kmod + 1 + o;
                    sl = sl >= W ? sl - W : sl;
                    ent[buf][base + sl] = fifo[s][it];
                }
            }
            lds_barrier();
            T piv = ubuf[buf][kmod];
            if (!(fabs((double)piv) > 0.0) || !isfinite((double)piv)) { bad = 1; piv = T(1); }
            const T inv = T(1) / piv;
            if (tid == 0) { mon.d(inv); mon.u(piv); }
            const int kl = k * ldf, rl = (n - 1 - k) * ldf + fac_pos(rk, nrf);
#pragma unroll
            for (int it = 0; it < NI; ++it) {
                const bool isl = qq[it] < W;
                const int o = isl ? qq[it] : qq[it] - W;
                int sl = kmod + o;
                sl = sl >= W ? sl - W : sl;
                const T lv = lbuf[buf][sl] * inv;
                const T uv = o == 0 ? inv : ubuf[buf][sl] * inv;
                T *ldst = Lr + (kl + fac_pos(srot[it], nrf));
                T *udst = o == 0 ? Di + k : Ur + (rl + soff[it]);
                T *dst = k < send[it] ? (isl ? ldst : udst) : dummy + it;
                *dst = isl ? lv : uv;
                mon.u(!isl && o != 0 && k < send[it] ? ubuf[buf][sl] : T(0));
                srot[it] = srot[it] + 1 == R ? 0 : srot[it] + 1;
            }
            rk = rk == 0 ? R - 1 : rk - 1;
            T l[RB], u[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i) l[i] = lbuf[buf][tr * RB + i] * inv;
#pragma unroll
            for (int jj = 0; jj < RB; ++jj) u[jj] = ubuf[buf][tc * RB + jj];
            T er[RB], ec[RB];
            if (orow) {
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) er[jj] = ent[buf][tc * RB + jj];
            }
            if (ocol) {
#pragma unroll
                for (int i = 0; i < RB; ++i) ec[i] = ent[buf][W + tr * RB + i];
            }
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int jj = 0; jj < RB; ++jj) {
                    T v = a[i][jj] - l[i] * u[jj];
                    if (i == ps) v = orow ? er[jj] : v;
                    if (jj == ps) v = ocol ? ec[i] : v;
                    a[i][jj] = v;
                }
            const int kf = k + U, kfl = kf * ld;
#pragma unroll
            for (int it = 0; it < NI; ++it) {
                fifo[s][it] = *(kf < fend[it] ? M + (kfl + foff[it]) : B.zero);
                mon.a(fifo[s][it]);
            }
        }
        kw += U;
        kw = kw == W ? 0 : kw;
    }
    if (bad && tid == 0) atomicOr(B.flags, 4);
    lu_monitor_finish<T, (NT + 63) / 64>(mon, B);
}

// value of v in lane `lane` of the wavefront (uniform lane index)
template <typename T>
__device__ __forceinline__ T wave_bcast(T v, int lane);
template <>
__device__ __forceinline__ float wave_bcast<float>(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <>
__device__ __forceinline__ double wave_bcast<double>(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}
// value of v in lane J of each row of 16 lanes (DPP row broadcast, no SGPR
// round trip)
template <int J>
__device__ __forceinline__ float row_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + J, 0xF, 0xF, true));
}
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x150 + J, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + J, 0xF, 0xF, true);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Elimination step J of a 16 x 16 tile held by rows (lane l: row l mod 16, the
// four rows of 16 lanes identical): multipliers stored below the diagonal,
// the reciprocal of pivot J kept in lane J of dinv.
template <int J, typename T>
__device__ __forceinline__ void tile_lu_step(T (&d)[16], int lc, int lane, T &dinv) {
    const T piv = row_bcast<J>(d[J]);
    const T dj = lc > J ? d[J] : T(0);          // masked before the reciprocal is known
    T inv;
    if constexpr (sizeof(T) == 4) {
        // the hardware reciprocal (1 ulp): the chain from one pivot to the
        // next is broadcast, reciprocal, multiply, FMA; the refinement sweeps
        // absorb the factor's rounding
        inv = __builtin_amdgcn_rcpf(piv);
    } else {
        inv = __builtin_amdgcn_rcp(piv);            // then two Newton steps
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
    }
    dinv = lane == J ? inv : dinv;
    const T lm = dj * inv;
#pragma unroll
    for (int c = J + 1; c < 16; ++c) d[c] = fma(-lm, row_bcast<J>(d[c]), d[c]);
    d[J] = lc > J ? lm : d[J];
}
template <typename T, int... J>
__device__ __forceinline__ void tile_lu(T (&d)[16], int lc, int lane, T &dinv, std::integer_sequence<int, J...>) {
    (tile_lu_step<J>(d, lc, lane, dinv), ...);
}

// ---------------------------------------------------------------------------
// Blocked band LU without pivoting on the matrix cores (MFMA 16x16x4).
// The window of W = 16 TT rows and columns (W >= bw + 16) is split into
// 16 x 16 tiles held in MFMA accumulators, tile (I, J) by wavefront
// (I TT + J) mod NW.  Tile slots are circular like the rows: global row i sits
// in slot i mod W, so panel p (columns 16p .. 16p+15) is tile column and tile
// row P = p mod TT and no data moves between registers when the window
// advances.  Per panel:
//   1. the panel tile row and column go to LDS, and their accumulators are
//      refilled with the entering rows / columns of the next window (loads
//      that have the panel factorisation to arrive);
//   2. a writer wavefront factors the diagonal tile (L11 U11);
//   3. the writers solve l U11 = a for every other row of the tile column and
//      L11 u = a for every other column of the tile row, one thread each;
//   4. the writers store L and U of the panel in the solves' factor layout
//      while
//   5. the NW tile wavefronts take C -= L(I, P) U(P, J) on every other tile as
//      four MFMA steps.
// Tile and writer wavefronts (LU_NS of them, holding no tiles) run separate
// loops with the same barriers.  The tile wavefronts issue only loads and the
// writers only stores, so no wait for a load ever waits for a store (the
// memory counter is shared by both, in order, per wavefront), and the writers'
// registers are free of the window.  The arithmetic is that of the unblocked
// elimination in a different order.
// ---------------------------------------------------------------------------
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // accumulator register r of lane l holds tile row crow(l, r), column l mod 16
    static __device__ __forceinline__ int crow(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ int crow(int l, int r) { return (l >> 4) + 4 * r; }
};

constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }
constexpr int LU_NS = 5;           // writer wavefronts of the blocked factorisation

template <typename T, int TT, int NW>
__global__ __launch_bounds__(64 * (NW + LU_NS)) void k_band_lu_mfma(BandArgs<T> B) {
    typedef typename Mfma<T>::v4 v4;
    constexpr int W = 16 * TT, NTILE = TT * TT, MT = (NTILE + NW - 1) / NW;
    static_assert(2 * (W - 16) <= 64 * LU_NS, "one writer thread per panel row and column");
    const BandSys Sy = B.sys[blockIdx.x];
    if (B.skip && B.skip[blockIdx.x]) return;
    const int n = Sy.n, bw = Sy.bw, ld = 2 * bw + 1;
    const int ws = bw > 0 ? bw : 1, ldf = Sy.ldf, nrf = ldf >> 6, R = ldf;
    const T *M = B.band + Sy.off;
    __shared__ T Pc[W][17];        // panel tile column by row slot (L11\U11 in the diagonal tile, then L21)
    __shared__ T Pr[16][W + 1];    // panel tile row by column slot (then U12)
    __shared__ T dinv[16];
    // the wavefront index is uniform: keep tile coordinates and branches scalar
    const int tid = threadIdx.x, wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, lc = lane & 15;
    const int npan = (n + 15) / 16;
    LuMon mon;
    if (wv < NW) {
        // ---- tile wavefronts: hold the window, refill it, apply the trailing updates
        v4 acc[MT];
        auto base_of = [](int S, int P, int k0) { return k0 + 16 * ((S - P + TT) % TT); };
        // tile (I, J) of the window whose panel starts at k0 (slot P), from the
        // band: outside the band zero, beyond n the identity (pivots 1)
#define LP_TILE_LOAD(DST_, I_, J_, P_, K0_)                                                    \
        do {                                                                                  \
            const int gi0 = base_of(I_, P_, K0_), gj = base_of(J_, P_, K0_) + lc;             \
            _Pragma("unroll") for (int r = 0; r < 4; ++r) {                                    \
                const int gi = gi0 + Mfma<T>::crow(lane, r), d = gi - gj;                      \
                const bool in = gi < n && gj < n && d <= bw && d >= -bw;                       \
                const T *src = in ? M + ((long long)gj * ld + d + bw) : (gi == gj ? B.one : B.zero); \
                DST_[r] = *src;                                                               \
                mon.a(in ? DST_[r] : T(0));     /* the identity padding is not the matrix's */ \
            }                                                                                 \
        } while (0)
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            const int q = wv + NW * t;
            if (q < NTILE) LP_TILE_LOAD(acc[t], q / TT, q % TT, 0, 0);
        }
        for (int p = 0; p < npan; ++p) {
            const int k0 = 16 * p, P = p % TT;
            // 1. panel tiles to LDS, then their accumulators refilled with the
            //    entering tiles (all writes first: a write that waits on the
            //    previous panel's loads must not also wait on these)
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const int q = wv + NW * t;
                if (q >= NTILE) continue;
                const int I = q / TT, J = q % TT;
                if (J == P) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) Pc[16 * I + Mfma<T>::crow(lane, r)][lc] = acc[t][r];
                } else if (I == P) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) Pr[Mfma<T>::crow(lane, r)][16 * J + lc] = acc[t][r];
                }
            }
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const int q = wv + NW * t;
                if (q >= NTILE) continue;
                const int I = q / TT, J = q % TT;
                if (I == P || J == P) LP_TILE_LOAD(acc[t], I, J, (P + 1) % TT, k0 + 16);
            }
            lds_barrier();                 // A: panel in LDS
            lds_barrier();                 // B: diagonal tile factored
            lds_barrier();                 // C: L21 and U12 ready
            // 5. trailing update of the other tiles: operands of two tiles at a time, then their MFMAs
#pragma unroll
            for (int t0 = 0; t0 < MT; t0 += 2) {
                T av[2][4], bv[2][4];
#pragma unroll
                for (int t = t0; t < t0 + 2 && t < MT; ++t) {
                    const int q = wv + NW * t;
                    const int I = q < NTILE ? q / TT : 0, J = q < NTILE ? q % TT : 0;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        av[t - t0][kk] = -Pc[16 * I + lc][4 * kk + (lane >> 4)];
                        bv[t - t0][kk] = Pr[4 * kk + (lane >> 4)][16 * J + lc];
                    }
                }
#pragma unroll
                for (int t = t0; t < t0 + 2 && t < MT; ++t) {
                    const int q = wv + NW * t;
                    if (q >= NTILE) continue;
                    const int I = q / TT, J = q % TT;
                    if (I == P || J == P) continue;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) acc[t] = Mfma<T>::op(av[t - t0][kk], bv[t - t0][kk], acc[t]);
                }
            }
            lds_barrier();                 // D: LDS free for the next panel
        }
#undef LP_TILE_LOAD
    } else {
        // ---- writer wavefronts: factor the panel and write L and U out
        const int wr = wv - NW, wt = tid - 64 * NW;     // writer wavefront / thread index
        T *Lr = B.fac + Sy.foff, *Ur = Lr + (long long)n * ldf, *Di = Ur + (long long)n * ldf;
        int bad = 0;
        for (int p = 0; p < npan; ++p) {
            const int k0 = 16 * p, P = p % TT;
            lds_barrier();                 // A
            // 2. diagonal tile: lanes 0..15 of writer 0 hold its rows
            if (wr == 0) {
                T d[16];
                const int rr = 16 * P + lc;
#pragma unroll
                for (int c = 0; c < 16; ++c) d[c] = Pc[rr][c];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    T piv = wave_bcast(d[j], j);
                    if (!(fabs((double)piv) > 0.0) || !isfinite((double)piv)) { bad = 1; piv = T(1); }
                    const T inv = T(1) / piv;
                    if (k0 + j < n) { mon.d(inv); mon.u(piv); }
                    if (lane == j) dinv[j] = inv;
                    const T l = d[j] * inv;
#pragma unroll
                    for (int c = j + 1; c < 16; ++c) {
                        const T u = wave_bcast(d[c], j);
                        d[c] = lc > j ? d[c] - l * u : d[c];
                    }
                    d[j] = lc > j ? l : d[j];
                }
                if (lane < 16) {
#pragma unroll
                    for (int c = 0; c < 16; ++c) Pc[rr][c] = d[c];
                }
            }
            lds_barrier();                 // B
            // 3. the other rows of the tile column (l U11 = a) and columns of the tile row (L11 u = a)
            if (wt < W - 16) {
                // one row, U11 rows streamed from LDS one row ahead
                const int rho = (16 * (P + 1) + wt) % W;
                T a[16], ur[16], un[16];
#pragma unroll
                for (int c = 0; c < 16; ++c) a[c] = Pc[rho][c];
#pragma unroll
                for (int c2 = 0; c2 < 16; ++c2) un[c2] = Pc[16 * P][c2];
                un[0] = dinv[0];
#pragma unroll
                for (int c = 0; c < 16; ++c) {
#pragma unroll
                    for (int c2 = c; c2 < 16; ++c2) ur[c2] = un[c2];
                    if (c + 1 < 16) {
#pragma unroll
                        for (int c2 = c + 2; c2 < 16; ++c2) un[c2] = Pc[16 * P + c + 1][c2];
                        un[c + 1] = dinv[c + 1];
                    }
                    a[c] *= ur[c];
#pragma unroll
                    for (int c2 = c + 1; c2 < 16; ++c2) a[c2] -= a[c] * ur[c2];
                }
#pragma unroll
                for (int c = 0; c < 16; ++c) Pc[rho][c] = a[c];
            } else if (wt < 2 * (W - 16)) {
                // one column (unit lower L11), L11 columns streamed from LDS one ahead
                const int sig = (16 * (P + 1) + wt - (W - 16)) % W;
                T u[16], lr[16], ln[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) u[r] = Pr[r][sig];
#pragma unroll
                for (int r2 = 1; r2 < 16; ++r2) ln[r2] = Pc[16 * P + r2][0];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
#pragma unroll
                    for (int r2 = r + 1; r2 < 16; ++r2) lr[r2] = ln[r2];
                    if (r + 1 < 16) {
#pragma unroll
                        for (int r2 = r + 2; r2 < 16; ++r2) ln[r2] = Pc[16 * P + r2][r + 1];
                    }
#pragma unroll
                    for (int r2 = r + 1; r2 < 16; ++r2) u[r2] -= lr[r2] * u[r];
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) Pr[r][sig] = u[r];
            }
            lds_barrier();                 // C
            // 4. factors of columns / rows k0 .. k0+15 in the solves' layout, with
            //    fixed trip counts so that all LDS reads go out before the stores
            const int kr0 = k0 % R, rr0 = (n - 1 - k0) % R;     // k0 mod R, (n-1-k0) mod R
            {
                // L(k + o, k): column c = wr + LU_NS j, lanes over consecutive o
                constexpr int NC = (16 + LU_NS - 1) / LU_NS, NO = W / 64 + 1;
                T lv[NC][NO];
                long long la[NC][NO];
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const int c0 = wr + LU_NS * j, c = c0 < 16 ? c0 : 15, k = k0 + c;
                    int kmod = kr0 + c;                  // k mod R
                    kmod = kmod >= R ? kmod - R : kmod;
#pragma unroll
                    for (int u = 0; u < NO; ++u) {
                        const int o = lane + 1 + 64 * u, i = k + o;
                        const bool ok = c0 < 16 && o <= ws && k < n && i < n;
                        int sl = kmod + o;                   // (k + o) mod R
                        sl = sl >= R ? sl - R : sl;
                        int iw = 16 * P + c + o;
                        iw = iw >= W ? iw - W : iw;
                        lv[j][u] = ok ? Pc[iw][c] : T(0);
                        la[j][u] = ok ? (long long)k * ldf + fac_pos(sl, nrf) : -1;
                    }
                }
#pragma unroll
                for (int j = 0; j < NC; ++j)
#pragma unroll
                    for (int u = 0; u < NO; ++u)
                        if (la[j][u] >= 0) Lr[la[j][u]] = lv[j][u];
            }
            {
                // U(k0 + c, j), j = k0 + c + 1 .. k0 + c + bw: four columns j per
                // pass, lanes c = 0..15 over the panel rows
                constexpr int NJ = (W + 4 * LU_NS - 1) / (4 * LU_NS);
                const int c = lane & 15, k = k0 + c;
                int rk = rr0 - c;                        // (n-1-k) mod R
                rk = rk < 0 ? rk + R : rk;
                const int pk = fac_pos(rk, nrf);
                const T dk = dinv[c];
                T uvv[NJ];
                long long ua[NJ];
#pragma unroll
                for (int u = 0; u < NJ; ++u) {
                    const int jo = (lane >> 4) + 4 * wr + 4 * LU_NS * u;
                    const int j = k0 + 1 + jo;
                    const bool ok = jo < 15 + ws && j > k && j - k <= ws && j < n;
                    int jw = 16 * P + 1 + jo;
                    jw = jw >= W ? jw - W : jw;
                    jw = jw >= W ? jw - W : jw;
                    const T uval = ok ? (j < k0 + 16 ? Pc[16 * P + c][(j - k0) & 15] : Pr[c][jw]) : T(0);
                    mon.u(uval);
                    uvv[u] = uval * dk;
                    ua[u] = ok ? (long long)(n - 1 - j) * ldf + pk : -1;
                }
#pragma unroll
                for (int u = 0; u < NJ; ++u)
                    if (ua[u] >= 0) Ur[ua[u]] = uvv[u];
            }
            if (wr == 0 && lane < 16 && k0 + lane < n) Di[k0 + lane] = dinv[lane];
            lds_barrier();                 // D
        }
        if (bad && lane == 0) atomicOr(B.flags, 4);
    }
    lu_monitor_finish<T, NW + LU_NS>(mon, B);
}

// ---------------------------------------------------------------------------
// Blocked band LU with a one-panel lookahead.  Same window, tiles, elimination
// and factor layout as the kernel above; the order of the work differs:
//   tile wavefronts, panel p (window slot P, next slot P1):
//     L1. apply panel p to the tiles of slot row and column P1 only, write
//         them to the other LDS buffer (the raw panel p+1) and refill them;
//     L2. apply panel p to every other tile;
//     S.  store L and U of panel p (factored one panel earlier), after L2;
//   writer wavefronts, panel p:
//     F.  factor panel p+1 (after L1), alongside L2 and S.
// Each writer wavefront factors the 16 x 16 diagonal tile of the panel into
// its own LDS copy, so the writers never wait for one another: two barriers
// per panel.  Panel tiles sit in LDS by row with the elimination index
// permuted (index 4 kk + g at 4 g + kk) so that a lane of lane group g reads
// its four MFMA operands with one 16-byte access; the L21 block is kept
// negated (the update is C += (-L21) U12).  Each wavefront holds bit masks of
// its tiles by window slot row and column.
// ---------------------------------------------------------------------------
constexpr int LU_LDP = 20;                  // LDS row pitch of a panel (16 used)
__device__ __forceinline__ int lu_perm(int k) { return (k & 3) * 4 + (k >> 2); }

template <typename T>
struct alignas(16) Quad { T v[4]; };

template <typename T, int TT>
__global__ __launch_bounds__(64 * (TT + LU_NS)) void k_band_lu_la(BandArgs<T> B) {
    typedef typename Mfma<T>::v4 v4;
    // TT tile wavefronts; wavefront w holds tile t = 0..TT-1 at window slots
    // (t, (w + t) mod TT): one tile in every slot row and every slot column
    constexpr int NW = TT, W = 16 * TT, MT = TT;
    constexpr int NRF = solve_nr(W - 16);         // solve registers per lane of this window's bandwidths
    static_assert(2 * (W - 16) <= 64 * LU_NS, "one writer thread per panel row and column");
    const BandSys Sy = B.sys[blockIdx.x];
    if (B.skip && B.skip[blockIdx.x]) return;
    const int n = Sy.n, bw = Sy.bw, ld = 2 * bw + 1;
    const int ws = bw > 0 ? bw : 1, ldf = Sy.ldf;
    if (n <= 0) return;
    if (ldf != 64 * NRF || bw > W - 16) {          // layout not made for this window: report, write nothing
        if (threadIdx.x == 0) atomicOr(B.flags, 4);
        return;
    }
    const T *M = B.band + Sy.off;
    __shared__ Quad<T> PcQ[2][W][LU_LDP / 4];      // panel tile column by row slot (L21 negated)
    __shared__ Quad<T> PrQ[2][W][LU_LDP / 4];      // panel tile row by column slot (U12), transposed
    __shared__ Quad<T> DgQ[LU_NS][16][4];          // factored diagonal tile by rows, per writer wavefront
    __shared__ T Dt[LU_NS][16][16];                // the same by columns
    __shared__ T Dv[LU_NS][16];                    // pivot reciprocals
    __shared__ T Zs[1];                            // a zero, read by masked lanes
    __shared__ Quad<T> DgSQ[2][16][4];             // factored diagonal tile of panels of each parity (for the stores)
    __shared__ T DvS[2][16];
    T (*Pc)[W][LU_LDP] = reinterpret_cast<T (*)[W][LU_LDP]>(&PcQ[0][0][0]);
    T (*Pr)[W][LU_LDP] = reinterpret_cast<T (*)[W][LU_LDP]>(&PrQ[0][0][0]);
    T (*Dg)[16][16] = reinterpret_cast<T (*)[16][16]>(&DgQ[0][0][0]);
    T (*DgS)[16][16] = reinterpret_cast<T (*)[16][16]>(&DgSQ[0][0][0]);
    const int tid = threadIdx.x, wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, lc = lane & 15, lg = lane >> 4;
    const int npan = (n + 15) / 16;
    LuMon mon;
    T *Lr = B.fac + Sy.foff, *Ur = Lr + (long long)n * ldf, *Di = Ur + (long long)n * ldf;
    // L and U of panel ps from buffer bb in the solves' layout (fac_pos, R
    // slots per column), by worker w of NWK (its share of the columns and rows)
    constexpr int R = 64 * NRF;
    auto store = [&](int ps, int bb, int w, auto nwk) {
        constexpr int NWK = decltype(nwk)::value;
        const int k0 = 16 * ps, P = ps % TT, q = ps & 1;
        const int kr0 = (k0 + 1) % R, rr0 = (n - 1 - k0) % R;   // (k0 + 1) mod R, (n - 1 - k0) mod R
        struct Grp { T v[NRF]; };
        // L: column c = w + NWK j; lane l, register m holds slot
        // 32 (2m + l / 32) + l mod 32 (one vector store per lane)
#pragma unroll
        for (int j = 0; j < (16 + NWK - 1) / NWK; ++j) {
            const int c = w + NWK * j, k = k0 + c;
            if (c >= 16 || k >= n) break;
            int k1 = kr0 + c;                             // (k + 1) mod R
            k1 = k1 >= R ? k1 - R : k1;
            Grp gv;
#pragma unroll
            for (int m = 0; m < NRF; ++m) {
                const int s = 32 * (2 * m + (lane >> 5)) + (lane & 31);
                int o = s - k1;
                o = o < 0 ? o + R : o;
                o += 1;                                   // row k + o with (k + o) mod R = s, 1 <= o <= R
                const int dr = c + o;
                int iw = 16 * P + dr;
                iw = iw >= W ? iw - W : iw;
                const bool ok = o <= ws && k + o < n;
                // one unconditional LDS read: L11 from the copy, -L21 from the panel, else zero
                const T *src = dr < 16 ? &DgS[q][dr & 15][c] : &Pc[bb][iw][lu_perm(c)];
                src = ok ? src : &Zs[0];
                const T v = *src;
                gv.v[m] = dr < 16 ? v : -v;
            }
            *reinterpret_cast<Grp *>(Lr + (long long)k * ldf + lane * NRF) = gv;
        }
        // U(k0 + c, j) / U(k0 + c, k0 + c), j = k0 + c + 1 .. k0 + c + ws:
        // lanes c = 0..15 over the panel rows, four columns per pass
        {
            constexpr int NJ = (W + 4 * NWK - 1) / (4 * NWK);
            const int c = lc, k = k0 + c;
            int rk = rr0 - c;                             // (n - 1 - k) mod R
            rk = rk < 0 ? rk + R : rk;
            const int pk = fac_pos(rk, NRF);
            const T dk = DvS[q][c];
#pragma unroll
            for (int u = 0; u < NJ; ++u) {
                const int jo = lg + 4 * w + 4 * NWK * u;
                const int j = k0 + 1 + jo;
                const bool ok = jo < 15 + ws && j > k && j - k <= ws && j < n;
                int jw = 16 * P + 1 + jo;
                jw = jw >= W ? jw - W : jw;
                jw = jw >= W ? jw - W : jw;
                const int dj = j - k0;
                const T *src = dj < 16 ? &DgS[q][c][dj & 15] : &Pr[bb][jw][lu_perm(c)];
                const T v = *src;
                mon.u(ok ? v : T(0));
                if (ok) Ur[(long long)(n - 1 - j) * ldf + pk] = v * dk;
            }
        }
        if (w == 0 && lane < 16 && k0 + lane < n) Di[k0 + lane] = DvS[q][lane];
    };
    if (wv < NW) {
        // ---- tile wavefronts
        v4 acc[MT];
        auto base_of = [](int S, int P, int k0) { return k0 + 16 * ((S - P + TT) % TT); };
        auto col_of = [&](int t) { return wv + t < TT ? wv + t : wv + t - TT; };
        // bits of this wavefront's tiles in slot row S (tile S) and column S
        auto rmask = [&](int S) { return 1u << S; };
        auto cmask = [&](int S) { return 1u << (S >= wv ? S - wv : S - wv + TT); };
        // tile (I, J) of the window whose panel starts at K0 (slot P), from the
        // band: outside the band zero, beyond n the identity
#define LP_TILE_LOAD(DST_, I_, J_, P_, K0_)                                                    \
        do {                                                                                  \
            const int gi0 = base_of(I_, P_, K0_), gj = base_of(J_, P_, K0_) + lc;             \
            _Pragma("unroll") for (int r = 0; r < 4; ++r) {                                    \
                const int gi = gi0 + Mfma<T>::crow(lane, r), d = gi - gj;                      \
                const bool in = gi < n && gj < n && d <= bw && d >= -bw;                       \
                const T *src = in ? M + ((long long)gj * ld + d + bw) : (gi == gj ? B.one : B.zero); \
                DST_[r] = *src;                                                               \
                mon.a(in ? DST_[r] : T(0));     /* the identity padding is not the matrix's */ \
            }                                                                                 \
        } while (0)
        // entering tiles in flight: staging registers, filled by loads from
        // clamped (always valid) band addresses; out-of-band and beyond-n
        // elements are set when the tile reaches its accumulator
        constexpr int NSTG = 2;
        T stg[NSTG][4];
        int loff[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) loff[r] = lc * (ld - 1) + Mfma<T>::crow(lane, r);
        const int nld = n * ld;
        auto inside = [&](int gi0, int gj0) {
            return gi0 - gj0 <= bw - 15 && gj0 - gi0 <= bw - 15 && gi0 + 15 < n && gj0 + 15 < n;
        };
        // slot PN tiles (the column tile first) to buffer BB, then their
        // replacements, entering when the panel at K0N leaves the window, into
        // the staging registers (they reach the accumulators one panel later)
#define LP_EMIT(PN, BB, K0N)                                                                   \
        do {                                                                                  \
            const unsigned cmk = cmask(PN), rmk = rmask(PN);                                  \
            _Pragma("unroll") for (int t = 0; t < MT; ++t) {                                   \
                const int I = t, J = col_of(t);                                               \
                if ((cmk >> t) & 1) {                                                         \
                    _Pragma("unroll") for (int r = 0; r < 4; ++r)                              \
                        Pc[BB][16 * I + Mfma<T>::crow(lane, r)][lu_perm(lc)] = acc[t][r];     \
                } else if ((rmk >> t) & 1) {                                                  \
                    _Pragma("unroll") for (int r = 0; r < 4; ++r)                              \
                        Pr[BB][16 * J + lc][lu_perm(Mfma<T>::crow(lane, r))] = acc[t][r];     \
                }                                                                             \
            }                                                                                 \
            const int PN2 = (PN) + 1 == TT ? 0 : (PN) + 1;                                    \
            unsigned emk = cmk | rmk;                                                         \
            _Pragma("unroll") for (int si = 0; si < NSTG; ++si) {                              \
                if (emk == 0) break;                                                          \
                const int t = __builtin_ctz(emk);                                             \
                emk &= emk - 1u;                                                              \
                const int gi0 = base_of(t, PN2, (K0N) + 16), gj0 = base_of(col_of(t), PN2, (K0N) + 16); \
                const int b0 = gj0 * ld + gi0 - gj0 + bw;                                     \
                _Pragma("unroll") for (int r = 0; r < 4; ++r)                                  \
                    stg[si][r] = M[min(max(b0 + loff[r], 0), nld - 1)];                       \
            }                                                                                 \
        } while (0)
        // the tiles of slot PN staged one panel ago (when the window's panel
        // slot was PS at K0S) into their accumulators
#define LP_ARRIVE(PN, PS, K0S)                                                                 \
        do {                                                                                  \
            const unsigned amk = cmask(PN) | rmask(PN);                                       \
            _Pragma("unroll") for (int t = 0; t < MT; ++t) {                                   \
                if ((amk >> t) & 1) {                                                         \
                    const bool second = (amk & ((1u << t) - 1u)) != 0;                        \
                    const int gi0 = base_of(t, PS, K0S), gj0 = base_of(col_of(t), PS, K0S);   \
                    _Pragma("unroll") for (int r = 0; r < 4; ++r) acc[t][r] = second ? stg[1][r] : stg[0][r]; \
                    if (!inside(gi0, gj0)) {                                                  \
                        const int gj = gj0 + lc;                                              \
                        _Pragma("unroll") for (int r = 0; r < 4; ++r) {                        \
                            const int gi = gi0 + Mfma<T>::crow(lane, r), d = gi - gj;          \
                            const bool in = gi < n && gj < n && d <= bw && d >= -bw;           \
                            acc[t][r] = in ? acc[t][r] : (gi == gj ? T(1) : T(0));            \
                            mon.a(in ? acc[t][r] : T(0));                                     \
                        }                                                                     \
                    } else {                                                                  \
                        _Pragma("unroll") for (int r = 0; r < 4; ++r) mon.a(acc[t][r]);        \
                    }                                                                         \
                }                                                                             \
            }                                                                                 \
        } while (0)
        // C += (-L21) U12 from buffer BB on the tiles in MASK, operands of two
        // tiles at a time
#define LP_UPDATE(BB, MASK)                                                                    \
        do {                                                                                  \
            _Pragma("unroll") for (int t0 = 0; t0 < MT; t0 += 2) {                             \
                if ((((MASK) >> t0) & 3u) == 0) continue;                                     \
                Quad<T> av[2], bv[2];                                                         \
                _Pragma("unroll") for (int t = t0; t < t0 + 2 && t < MT; ++t) {                \
                    av[t - t0] = PcQ[BB][16 * t + lc][lg];                                    \
                    bv[t - t0] = PrQ[BB][16 * col_of(t) + lc][lg];                            \
                }                                                                             \
                _Pragma("unroll") for (int t = t0; t < t0 + 2 && t < MT; ++t) {                \
                    if (!(((MASK) >> t) & 1)) continue;                                       \
                    _Pragma("unroll") for (int kk = 0; kk < 4; ++kk)                           \
                        acc[t] = Mfma<T>::op(av[t - t0].v[kk], bv[t - t0].v[kk], acc[t]);     \
                }                                                                             \
            }                                                                                 \
        } while (0)
#pragma unroll
        for (int t = 0; t < MT; ++t) LP_TILE_LOAD(acc[t], t, col_of(t), 0, 0);
        LP_EMIT(0, 0, 0);
        lds_barrier();                     // raw panel 0 in buffer 0
        lds_barrier();                     // panel 0 factored
        const unsigned valid = (1u << MT) - 1u;
        for (int p = 0; p + 1 < npan; ++p) {
            const int k0 = 16 * p, P = p % TT, P1 = P + 1 == TT ? 0 : P + 1, b = p & 1;
            const unsigned mP = cmask(P) | rmask(P), mP1 = cmask(P1) | rmask(P1);
            LP_ARRIVE(P, P1, k0 + 16);
            LP_UPDATE(b, mP1 & ~mP);                          // L1
            LP_EMIT(P1, b ^ 1, k0 + 16);
            lds_barrier();                 // A: raw panel p+1 in buffer b^1
            LP_UPDATE(b, valid & ~(mP | mP1));                // L2
            store(p, b, wv, std::integral_constant<int, NW>());   // the factors of panel p
            lds_barrier();                 // D: panel p+1 factored, buffer b free
        }
        store(npan - 1, (npan - 1) & 1, wv, std::integral_constant<int, NW>());
#undef LP_TILE_LOAD
#undef LP_EMIT
#undef LP_ARRIVE
#undef LP_UPDATE
    } else {
        // ---- writer wavefronts
        const int wr = wv - NW, wt = tid - 64 * NW;
        int bad = 0;
        // The writers' elimination is the panel's critical path and shares
        // its SIMDs with tile wavefronts doing the off-path trailing update and
        // stores: their instructions go first.
        __builtin_amdgcn_s_setprio(3);
        // Factor panel pf (raw in buffer bb): every writer wavefront factors
        // the diagonal tile itself (lane l < 16 holds row l), then lane wt
        // solves one L21 row (l U11 = a, stored negated) or one U12 column
        // (L11 u = a).  Both are the same forward substitution over a row of
        // 16 values read from this wavefront's copy of the tile: row c of U11
        // for the L21 rows (then scaled by 1 / U(c, c)), column c of L11 for
        // the U12 columns, so no wavefront diverges between the two.
        auto factor = [&](int pf, int bb) {
            const int P = pf % TT;
            T dinv = T(0);
            {
                T d[16];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const Quad<T> x = PcQ[bb][16 * P + lc][g];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) d[4 * kk + g] = x.v[kk];
                }
                tile_lu(d, lc, lane, dinv, std::make_integer_sequence<int, 16>());
                // a zero or non-finite pivot leaves a zero or non-finite reciprocal; a
                // merely small one is judged against the matrix scale at the end
                if (lane < 16 && !(fabs((double)dinv) > 0.0 && isfinite((double)dinv))) bad = 1;
                if (lane < 16 && 16 * pf + lane < n) { mon.d(dinv); mon.u(T(1) / dinv); }
                if (lane < 16) {
                    Dv[wr][lane] = dinv;
                    if (wr == 0) DvS[pf & 1][lane] = dinv;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        Quad<T> x;
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) x.v[kk] = d[4 * g + kk];
                        DgQ[wr][lc][g] = x;
                        if (wr == 0) DgSQ[pf & 1][lc][g] = x;
                    }
#pragma unroll
                    for (int c = 0; c < 16; ++c) Dt[wr][c][lc] = d[c];
                }
            }
            // the copy is read back by other lanes of this wavefront only
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
            if (wt < 2 * (W - 16)) {
                const bool isrow = wt < W - 16;
                const int idx = (16 * (P + 1) + (isrow ? wt : wt - (W - 16))) % W;
                Quad<T> *io = isrow ? &PcQ[bb][idx][0] : &PrQ[bb][idx][0];
                const Quad<T> *mq = isrow ? &DgQ[wr][0][0] : reinterpret_cast<const Quad<T> *>(&Dt[wr][0][0]);
                T x[16];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const Quad<T> v = io[g];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) x[4 * kk + g] = v.v[kk];
                }
                // row c + 1 is read while step c runs (the scheduling barriers
                // keep the reads from being hoisted all at once)
                Quad<T> m[2][4];
#pragma unroll
                for (int g = 0; g < 4; ++g) m[0][g] = mq[g];
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    if (c + 1 < 15) {
#pragma unroll
                        for (int g = 0; g < 4; ++g) m[(c + 1) & 1][g] = mq[4 * (c + 1) + g];
                    }
                    const T sc = wave_bcast(dinv, c);
                    x[c] *= isrow ? sc : T(1);
                    if (c + 1 < 16) {
#pragma unroll
                        for (int c2 = c + 1; c2 < 16; ++c2) x[c2] = fma(-x[c], m[c & 1][c2 >> 2].v[c2 & 3], x[c2]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                const T sg = isrow ? T(-1) : T(1);
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    Quad<T> v;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) v.v[kk] = sg * x[4 * kk + g];
                    io[g] = v;
                }
            }
        };
        if (wt == 0) Zs[0] = T(0);
        lds_barrier();                     // raw panel 0 in buffer 0
        factor(0, 0);
        lds_barrier();                     // panel 0 factored
        for (int p = 0; p + 1 < npan; ++p) {
            const int b = p & 1;
            lds_barrier();                 // A
            factor(p + 1, b ^ 1);
            lds_barrier();                 // D
        }
        if (bad && lane == 0) atomicOr(B.flags, 4);
    }
    lu_monitor_finish<T, TT + LU_NS>(mon, B);
}

// ---------------------------------------------------------------------------
// Band triangular solves, one wavefront per right-hand side: L y = r (unit
// lower), z = D^-1 y, then U' d = z with U' = D^-1 U (unit upper), x += d.
// The second is the first on reversed indices (row i -> n-1-i), so one pass
// routine serves both: a unit lower band solve over columns 0 .. n-1.
//
// The pass keeps R = 64 NR rows in NR registers per lane, in 2 NR halves of
// 32 rows (the slot map of fac_pos).  Columns go in blocks of 32; the rows of
// block b sit in half b mod 2NR, so with the block loop unrolled 2NR times the
// half holding the current rows is static: column k costs one broadcast of
// row k (readlane), NR FMAs on the window and one vector load of column k+D.
// Rows at or above k hold a zero coefficient in column k, so after its 32
// columns a block's half holds its finished values: they go to LDS and the
// half is refilled with the rows R further on.  The column index is clamped
// at n-1, whose column is zero (no row below n-1), and rows at or past n are
// zero, so the last block and the prefetch run straight through.
// ---------------------------------------------------------------------------
// LDS pad (rows) on each side of the right-hand side: a window and a
// super-block of blocks beyond the end (rows read past n are zero), for NR
// window registers per lane
constexpr int solve_pad(int nr) { return 128 * nr + 64; }
// rows per lane in flight when moving the right-hand side and the solution
constexpr int SOLVE_LD = 8;

// NR consecutive values of T at byte offset voff + soff of a buffer resource
// (raw buffer load: the column offset rides in an SGPR, the lane offset in a
// loop-invariant VGPR, so a column costs no vector address arithmetic)
template <typename T, int NR>
__device__ __forceinline__ void col_load(__amdgpu_buffer_rsrc_t rs, int voff, int soff, T (&dst)[NR]) {
    constexpr int NB = NR * (int)sizeof(T);
    unsigned w[NB / 4];
    if constexpr (NB == 8) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0);
        w[0] = v[0]; w[1] = v[1];
    } else if constexpr (NB == 12) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b96(rs, voff, soff, 0);
        w[0] = v[0]; w[1] = v[1]; w[2] = v[2];
    } else if constexpr (NB == 16) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
        w[0] = v[0]; w[1] = v[1]; w[2] = v[2]; w[3] = v[3];
    } else if constexpr (NB == 32) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
        const auto u = __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16, soff, 0);
        w[0] = v[0]; w[1] = v[1]; w[2] = v[2]; w[3] = v[3]; w[4] = u[0]; w[5] = u[1]; w[6] = u[2]; w[7] = u[3];
    } else {
        static_assert(NB == 24, "two to four values per lane");
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(rs, voff + 16, soff, 0);
        w[0] = v[0]; w[1] = v[1]; w[2] = v[2]; w[3] = v[3]; w[4] = u[0]; w[5] = u[1];
    }
    __builtin_memcpy(dst, w, NB);
}

template <typename T, int NR, int D, bool REV>
__device__ __forceinline__ void band_pass(const T *C, int n, int ldf, T *ys, int lane) {
    constexpr int H = 2 * NR, R = 64 * NR;
    // column k sits in ring slot k mod D, static within the unrolled super-block
    static_assert((32 * H) % D == 0, "prefetch ring divides a super-block");
    struct Grp { T v[NR]; };
    // row r of the pass (reversed rows for the second pass) in LDS
    auto yat = [&](int r) -> T & { return REV ? ys[n - 1 - r] : ys[r]; };
    T win[NR], cf[D][NR];
    // slot of (register m, this lane): rows s, s + R, ... in turn
#pragma unroll
    for (int m = 0; m < NR; ++m) win[m] = yat(32 * (2 * m + (lane >> 5)) + (lane & 31));
    const int nb = (n + 31) >> 5;
    // the resource from wavefront-uniform values (scalar registers)
    const unsigned long long cb = reinterpret_cast<unsigned long long>(C);
    const unsigned long long cu = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(cb >> 32)) << 32) |
                                  (unsigned)__builtin_amdgcn_readfirstlane((unsigned)cb);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(cu), (short)0,
                                                                         __builtin_amdgcn_readfirstlane(n * ldf * (int)sizeof(T)),
                                                                         0x00020000);
    const int voff = lane * NR * (int)sizeof(T);
#define LP_COL(KK, S) col_load<T, NR>(rs, voff, min((KK), n - 1) * ldf * (int)sizeof(T), cf[S])
#pragma unroll
    for (int s = 0; s < D; ++s) {
        LP_COL(s, s);
        __builtin_amdgcn_sched_barrier(0);   // issue in the loop body's order
    }
    for (int b0 = 0; b0 < nb; b0 += H) {
#pragma unroll
        for (int hb = 0; hb < H; ++hb) {
            // block b = b0 + hb in half hb: register hb / 2, lanes 32 (hb % 2) ..
            const int b = b0 + hb;
            const int mh = hb >> 1, lh = (hb & 1) << 5;
            const T ent = yat(32 * (b + H) + (lane & 31));      // the rows entering this half next
#pragma unroll
            for (int s = 0; s < 32; ++s) {
                const int sl = (32 * hb + s) % D;
                const T yk = wave_bcast(win[mh], lh + s);
                win[mh] = fma(-cf[sl][mh], yk, win[mh]);      // the half the next broadcast reads first
#pragma unroll
                for (int m = 0; m < NR; ++m)
                    if (m != mh) win[m] = fma(-cf[sl][m], yk, win[m]);
                // every column's updates happen in its column (otherwise the
                // compiler defers the other halves' chains to the block end and
                // keeps all their factor registers alive): an empty statement
                // that reads and writes the window
#pragma unroll
                for (int m = 0; m < NR; ++m) asm volatile("" : "+v"(win[m]));
                LP_COL(32 * b + s + D, sl);
                __builtin_amdgcn_sched_barrier(0);              // keep each prefetch in its column
            }
            const bool mine = (lane & 32) == lh;
            const int r = 32 * b + (lane & 31);
            if (mine) yat(r) = win[mh];
            win[mh] = mine ? ent : win[mh];
        }
    }
#undef LP_COL
}

constexpr int SOLVE_THREADS = 64;
template <typename T, int NR, int D>
__global__ __launch_bounds__(SOLVE_THREADS) void k_band_solve(SolveArgs<T> A) {
    constexpr int PAD = solve_pad(NR);
    static_assert(64 * NR + 32 * 2 * NR <= PAD, "pad too small");
    // one wavefront whose speed is its instruction issue: it owns its SIMD
    own_simd<SOLVE_THREADS>();
    const int sysi = blockIdx.x, f = blockIdx.y;
    const BandSys Sy = A.sys[sysi];
    if (f >= Sy.nrhs) return;
    const int id = sysi * A.rhs_per_sys + f;
    if (A.skip && A.skip[sysi]) return;
    if (A.conv && A.conv[id]) return;
    extern __shared__ unsigned char smem_raw[];
    const int n = Sy.n;
    T *ys = reinterpret_cast<T *>(smem_raw) + PAD;          // r, then z, then d, by row
    const int ldf = Sy.ldf;
    const T *Lr = A.fac + Sy.foff + (long long)f * Sy.fstride;
    const T *Ur = Lr + (long long)n * ldf, *Di = Ur + (long long)n * ldf;
    const double *rg = A.r + Sy.vec + (long long)f * n;
    double *x = A.x + Sy.vec + (long long)f * n;
    const int lane = threadIdx.x;
    // the right-hand side into LDS, SOLVE_LD rows per lane in flight (clamped
    // unconditional loads, then masked stores; the pads are zero)
    for (int i0 = lane - PAD; i0 < n + PAD; i0 += 64 * SOLVE_LD) {
        double v[SOLVE_LD];
#pragma unroll
        for (int u = 0; u < SOLVE_LD; ++u) v[u] = rg[min(max(i0 + 64 * u, 0), n - 1)];
#pragma unroll
        for (int u = 0; u < SOLVE_LD; ++u) {
            const int i = i0 + 64 * u;
            if (i < n + PAD) ys[i] = (i >= 0 && i < n) ? (T)v[u] : T(0);
        }
    }
    __syncthreads();
    band_pass<T, NR, D, false>(Lr, n, ldf, ys, lane);
    __syncthreads();
    // z = D^-1 y between the passes (pivot reciprocals read from the factors,
    // so the LDS holds one vector only)
    for (int i0 = lane; i0 < n; i0 += 64 * SOLVE_LD) {
        T dv[SOLVE_LD];
#pragma unroll
        for (int u = 0; u < SOLVE_LD; ++u) dv[u] = Di[min(i0 + 64 * u, n - 1)];
#pragma unroll
        for (int u = 0; u < SOLVE_LD; ++u) {
            const int i = i0 + 64 * u;
            if (i < n) ys[i] = ys[i] * dv[u];
        }
    }
    __syncthreads();
    band_pass<T, NR, D, true>(Ur, n, ldf, ys, lane);
    __syncthreads();
    if (A.assign) {
        for (int i = lane; i < n; i += 64) x[i] = (double)ys[i];
    } else {
        for (int i0 = lane; i0 < n; i0 += 64 * SOLVE_LD) {
            double v[SOLVE_LD];
#pragma unroll
            for (int u = 0; u < SOLVE_LD; ++u) v[u] = x[min(i0 + 64 * u, n - 1)];
#pragma unroll
            for (int u = 0; u < SOLVE_LD; ++u) {
                const int i = i0 + 64 * u;
                if (i < n) x[i] = v[u] + (double)ys[i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Dense application of explicit inverses (the small coarse systems): for each
// system s, x_s = Ainv_s b_s with Ainv_s column-major, Ainv_s[f n + i].  A block
// covers 64 rows; its 16 wavefronts split the columns (each a contiguous
// range, eight loads in flight per lane) and their partial sums are added in
// wavefront order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dense_rows(const DenseArgs &A, int s, int bx) {
    const int n = A.n;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = bx * 64 + lane;
    const int ic = i < n ? i : n - 1;
    const double *inv = A.inv + (long long)s * n * n + ic;
    const double *b = A.b + (long long)s * n;
    const int f0 = (n * w) >> 4, f1 = (n * (w + 1)) >> 4;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int f = f0;
    for (; f + 8 <= f1; f += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += inv[(long long)(f + u) * n] * b[f + u];
    }
    for (; f < f1; ++f) acc[0] += inv[(long long)f * n] * b[f];
    const double a = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __shared__ double red[16][64];
    red[w][lane] = a;
    __syncthreads();
    if (w == 0 && i < n) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += red[k][lane];
        A.x[(long long)s * n + i] = t;
    }
}
__global__ __launch_bounds__(1024) void k_dense_apply(DenseArgs A) {
    if (A.skip && A.skip[blockIdx.y]) return;
    dense_rows(A, blockIdx.y, blockIdx.x);
}

// true in the one block that finishes last (all blocks' global writes are
// then visible to it); the ticket is reset for the next launch
__device__ __forceinline__ bool last_block(int *ticket, int nb) {
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        last = atomicAdd(ticket, 1) == nb - 1;
        if (last) *ticket = 0;
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// ---------------------------------------------------------------------------
// Partition-of-unity merge (Algorithm 3 Step 4): x_h = Pi_h x_H + sum_j w_j e_j
// over the closed cores containing the node, ascending j.
// ---------------------------------------------------------------------------
// both regions in one launch (grid row = region)
__global__ void k_merge(MergeArgs Ap, MergeArgs Ac) {
    const MergeArgs &A = blockIdx.y == 0 ? Ap : Ac;
    const long long zo = blockIdx.z * A.zs;          // the sample's base and output fields
    const int sys0 = blockIdx.z * A.nper;            // and its systems
    const int n2 = 2 * A.N + 1, n1 = A.N + 1;
    const long long tot2 = (long long)n2 * n2, tot1 = (long long)n1 * n1;
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < tot2 + tot1; g += (long long)gridDim.x * blockDim.x) {
        const bool p1 = g >= tot2;
        const long long gg = p1 ? g - tot2 : g;
        const int nl = p1 ? n1 : n2;
        const int a = (int)(gg % nl), b = (int)(gg / nl);
        if (p1 && A.region == POROUS) continue;
        const int *lox = p1 ? A.own1_lo[0] : A.own2_lo[0], *cnx = p1 ? A.own1_n[0] : A.own2_n[0];
        const int *loy = p1 ? A.own1_lo[1] : A.own2_lo[1], *cny = p1 ? A.own1_n[1] : A.own2_n[1];
        const double w = 1.0 / (double)(cnx[a] * cny[b]);
        const int nf = p1 ? 1 : (A.region == POROUS ? 3 : 2);
        double acc[3];
        for (int f = 0; f < nf; ++f) acc[f] = p1 ? A.base1[zo + gg] : A.base[f][zo + gg];
        for (int ky = loy[b]; ky < loy[b] + cny[b]; ++ky)
            for (int kx = lox[a]; kx < lox[a] + cnx[a]; ++kx) {
                const SysDesc &S = A.sys[sys0 + kx + A.nsx * ky];
                if (p1) {
                    const int li = (a - S.x0) + S.lw1 * (b - S.y0);
                    acc[0] += w * A.e1[S.e1_off + li];
                } else {
                    const int li = (a - 2 * S.x0) + S.lw2 * (b - 2 * S.y0);
                    const long long nloc = (long long)S.lw2 * S.lh2;
                    for (int f = 0; f < nf; ++f) acc[f] += w * A.e2[S.e2_off + f * nloc + li];
                }
            }
        if (p1) A.out1[zo + gg] = acc[0];
        else for (int f = 0; f < nf; ++f) A.out[f][zo + gg] = acc[f];
    }
}

// lagged corrections from the merged field (LP_LAG_MERGED): block (system,
// region, sample) rewrites its local P2 lattice's corrections as the merged
// correction out - base of Step 4, zero on artificial nodes; on physical nodes
// every owner's correction is the same g - Pi_h x_H, so their merge is too
__global__ void k_lag_merged(MergeArgs Ap, MergeArgs Ac) {
    const MergeArgs &A = blockIdx.y == 0 ? Ap : Ac;
    if ((int)blockIdx.x >= A.nper) return;
    const long long zo = blockIdx.z * A.zs;
    const SysDesc &S = A.sys[blockIdx.z * A.nper + blockIdx.x];
    const int n2 = 2 * A.N + 1, nloc = S.lw2 * S.lh2;
    const int nf = A.region == POROUS ? 3 : 2;
    for (int q = threadIdx.x; q < nloc; q += blockDim.x) {
        const int a = q % S.lw2, b = q / S.lw2;
        const long long G = (2 * S.x0 + a) + (long long)n2 * (2 * S.y0 + b);
        const bool art = A.cls2[S.node_off + q] == 2;
        for (int f = 0; f < nf; ++f)
            A.e2w[S.e2_off + (long long)f * nloc + q] = art ? 0.0 : A.out[f][zo + G] - A.base[f][zo + G];
    }
}

// initial corrections e_j^0 = I_h x_0 - Pi_h x_H^0 on each local lattice, zero
// on artificial faces (the exact data is a(x) cos t, cos 0 = 1)
__global__ void k_init_corrections(InitArgs A) {
    const SysDesc S = A.sys[blockIdx.x];
    const int nloc = S.lw2 * S.lh2, ng = 2 * S.N + 1;
    const int nf = S.kind == KIND_POROUS ? 3 : 2;
    for (int q = threadIdx.x; q < nloc; q += blockDim.x) {
        const int a = q % S.lw2, b = q / S.lw2;
        const long long G = (2 * S.x0 + a) + (long long)ng * (2 * S.y0 + b);
        const int cls = A.cls2[S.node_off + q];
        for (int f = 0; f < nf; ++f)
            A.e[S.e2_off + (long long)f * nloc + q] = cls == 2 ? 0.0 : A.ex[f][G] - A.pro[f][S.zo + G];
    }
    if (S.kind == KIND_OSEEN)
        for (int v = threadIdx.x; v < S.lw1 * S.lh1; v += blockDim.x) A.e1[S.e1_off + v] = 0.0;
}

// Newton update of the coarse Navier-Stokes iterate: U += e, P += d, and the
// convergence test ||(e, d)|| <= tol ||(U, P)||, by the first 256 threads of
// a block (every thread of the block takes the barriers)
__device__ void newton_update_block(const NewtonArgs &A0, int smp) {
    constexpr int NT = 256;
    const int tid = threadIdx.x;
    const long long nu = A0.nu, np = A0.np, zo = smp * A0.zs;
    struct {
        double *U, *P;
        const double *e, *e1;
        int *done, *its;
        double tol;
    } A{A0.U + zo, A0.P + zo, A0.e + zo, A0.e1 + zo, A0.done + smp, A0.its + 2 * smp, A0.tol};
    double dd = 0.0, xx = 0.0;
    if (tid < NT) {
        for (long long i = tid; i < 2 * nu; i += NT) {
            const double u = A.U[i] + A.e[i];
            A.U[i] = u;
            dd += A.e[i] * A.e[i];
            xx += u * u;
        }
        for (long long i = tid; i < np; i += NT) {
            const double p = A.P[i] + A.e1[i];
            A.P[i] = p;
            dd += A.e1[i] * A.e1[i];
            xx += p * p;
        }
    }
    __shared__ double sd[NT], sx[NT];
    if (tid < NT) {
        sd[tid] = dd;
        sx[tid] = xx;
    }
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) { sd[tid] += sd[tid + s]; sx[tid] += sx[tid + s]; }
        __syncthreads();
    }
    if (tid == 0) {
        A.its[0] += 1;
        if (sqrt(sd[0]) <= A.tol * sqrt(sx[0])) *A.done = 1;
    }
}
__global__ __launch_bounds__(256) void k_newton_update(NewtonArgs A) {
    if (A.done[blockIdx.x]) return;
    newton_update_block(A, blockIdx.x);
}

// One chord step of the coarse Navier-Stokes solve after its right-hand side:
// x = J^-1 b by row blocks, then (last block) the correction to the node
// layout and the Newton update with its convergence test
__global__ __launch_bounds__(1024) void k_dense_newton(DenseNewtonArgs A) {
    const int smp = blockIdx.y;                   // one system per sample
    if (A.u.done[smp]) return;
    dense_rows(A.d, smp, blockIdx.x);
    if (!last_block(A.ticket + smp, gridDim.x)) return;
    oseen_finalize_rows(A.f, A.f.sys[smp], threadIdx.x, blockDim.x);
    __syncthreads();
    newton_update_block(A.u, smp);
}

// The three coarse porous solves: x_f = A_f^-1 b_f, then (last block) the
// solution to the node layout
__global__ __launch_bounds__(1024) void k_dense_porous(DensePorousArgs A) {
    const int smp = blockIdx.y / 3;               // three fields per sample
    dense_rows(A.d, blockIdx.y, blockIdx.x);
    if (!last_block(A.ticket + smp, gridDim.x * 3)) return;
    porous_finalize_rows(A.f, A.f.sys[smp], threadIdx.x, blockDim.x);
}

// start of the coarse Newton solve: the first iterate is the extrapolation
// of the previous levels (quadratic through three, linear through two at the
// second step, x^n at the first), counters reset (an unconverged previous step
// reported), and optionally a band cleared
__global__ void k_newton_start(NewtonStartArgs A) {
    const long long tot = A.nu2 + A.np;
    const int smp = blockIdx.y;
    const long long zo = smp * A.zs;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; blockIdx.y == 0 && i < A.band_n; i += (long long)gridDim.x * blockDim.x)
        A.band[i] = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot; i += (long long)gridDim.x * blockDim.x) {
        const bool u = i < A.nu2;
        const long long j = u ? i : i - A.nu2;
        // extrapolation through the last three levels (two at the second step)
        const long long jz = j + zo;
        const double x0 = u ? A.U0[jz] : A.P0[jz];
        const double xm = A.Um ? (u ? A.Um[jz] : A.Pm[jz]) : x0;
        const double x1 = A.Umm ? 3.0 * (x0 - xm) + (u ? A.Umm[jz] : A.Pmm[jz]) : 2.0 * x0 - xm;
        if (u) A.U1[jz] = x1;
        else A.P1[jz] = x1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // done starts at 1 (setup), so this reports the previous step only
        int *done = A.done + smp, *its = A.its + 2 * smp;
        if (*done == 0) atomicOr(A.flags, 2);
        its[1] = max(its[1], its[0]);
        *done = 0;
        *its = 0;
    }
}


// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static inline int grid_for(long long n, int block) {
    long long g = (n + block - 1) / block;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

void launch_prolong_p2(const ProlongArgs &a, int nsamples, hipStream_t st) {
    long long n = (long long)(2 * a.Nh + 1) * (2 * a.Nh + 1);
    hipLaunchKernelGGL(k_prolong_p2, dim3(grid_for(n, 256), nsamples), dim3(256), 0, st, a);
}
void launch_prolong_p1(const ProlongArgs &a, int nsamples, hipStream_t st) {
    long long n = (long long)(a.Nh + 1) * (a.Nh + 1);
    hipLaunchKernelGGL(k_prolong_p1, dim3(grid_for(n, 256), nsamples), dim3(256), 0, st, a);
}
int node_blocks(int maxnodes) { return maxnodes > 0 ? (maxnodes + GB - 1) / GB : 1; }

void launch_porous_rhs(const PorousArgs &a, int nsys, int maxnodes, int split, hipStream_t st) {
    if (split == 8) hipLaunchKernelGGL((k_porous_rhs<8>), dim3(node_blocks(8 * maxnodes), nsys), dim3(GB), 0, st, a);
    else hipLaunchKernelGGL((k_porous_rhs<1>), dim3(node_blocks(maxnodes), nsys), dim3(GB), 0, st, a);
}
void launch_porous_rhs_tiled(const PorousArgs &a, int nsys, int maxtiles, hipStream_t st) {
    hipLaunchKernelGGL(k_porous_rhs_tiled, dim3(maxtiles > 0 ? maxtiles : 1, nsys), dim3(256), 0, st, a);
}
void launch_porous_residual_tiled(const ResidualArgs &a, int nsys, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_porous_residual_tiled, dim3(blocks > 0 ? blocks : 1, nsys), dim3(256), 0, st, a);
}
void launch_porous_finalize(const FinalizeArgs &a, int nsys, int maxnodes, hipStream_t st) {
    hipLaunchKernelGGL(k_porous_finalize, dim3(node_blocks(maxnodes), nsys), dim3(GB), 0, st, a);
}
template <typename T>
void launch_porous_assemble(const AssembleArgs<T> &a, int nsys, hipStream_t st) {
    hipLaunchKernelGGL(k_porous_assemble<T>, dim3(nsys), dim3(256), 0, st, a);
}
void launch_oseen_rhs(const OseenArgs &a, int nsys, int maxnodes, int split, hipStream_t st) {
    if (split == 8) hipLaunchKernelGGL((k_oseen_rhs<8>), dim3(node_blocks(8 * maxnodes), nsys), dim3(GB), 0, st, a);
    else hipLaunchKernelGGL((k_oseen_rhs<1>), dim3(node_blocks(maxnodes), nsys), dim3(GB), 0, st, a);
}
template <typename T>
void launch_oseen_assemble(const OseenApplyArgs<T> &a, int nsys, int maxnodes, hipStream_t st) {
    hipLaunchKernelGGL((k_oseen_assemble<T>), dim3(node_blocks(maxnodes), nsys), dim3(GB), 0, st, a);
}
template <typename T>
void launch_oseen_rows(const OseenApplyArgs<T> &a, int nsys, int maxnodes, int maxbw, hipStream_t st) {
    hipLaunchKernelGGL((k_oseen_rows<T>), dim3(maxnodes, nsys), dim3(64), 3 * (2 * maxbw + 1) * sizeof(T), st, a);
}
void launch_oseen_rhs_tiled(const OseenArgs &a, int nsys, int maxtiles, hipStream_t st) {
    hipLaunchKernelGGL(k_oseen_rhs_tiled, dim3(maxtiles > 0 ? maxtiles : 1, nsys), dim3(256), 0, st, a);
}
void launch_oseen_residual_tiled(const OseenApplyArgs<double> &a, int nsys, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_oseen_residual_tiled, dim3(blocks > 0 ? blocks : 1, nsys), dim3(256), 0, st, a);
}
void launch_oseen_finalize(const FinalizeArgs &a, int nsys, int maxnodes, hipStream_t st) {
    hipLaunchKernelGGL(k_oseen_finalize, dim3(node_blocks(maxnodes), nsys), dim3(GB), 0, st, a);
}

template <typename T>
bool launch_band_lu(const BandArgs<T> &a, int nsys, int maxbw, int variant, hipStream_t st) {
    if (variant == 9 && maxbw <= 160) {
        // the same with a one-panel lookahead
        if (maxbw <= 64) { hipLaunchKernelGGL((k_band_lu_la<T, 5>), dim3(nsys), dim3(64 * (5 + LU_NS)), 0, st, a); return true; }
        if (maxbw <= 96) { hipLaunchKernelGGL((k_band_lu_la<T, 7>), dim3(nsys), dim3(64 * (7 + LU_NS)), 0, st, a); return true; }
        if (maxbw <= 128) { hipLaunchKernelGGL((k_band_lu_la<T, 9>), dim3(nsys), dim3(64 * (9 + LU_NS)), 0, st, a); return true; }
        if (maxbw <= 160) { hipLaunchKernelGGL((k_band_lu_la<T, 11>), dim3(nsys), dim3(64 * (11 + LU_NS)), 0, st, a); return true; }
        return false;
    }
    if (variant == 8 && maxbw <= 160) {
        // blocked factorisation on the matrix cores: window 16 TT >= bw + 16
        constexpr int X = 64 * LU_NS;
        if (maxbw <= 64) { hipLaunchKernelGGL((k_band_lu_mfma<T, 5, 4>), dim3(nsys), dim3(256 + X), 0, st, a); return true; }
        if (maxbw <= 96) { hipLaunchKernelGGL((k_band_lu_mfma<T, 7, 8>), dim3(nsys), dim3(512 + X), 0, st, a); return true; }
        if (maxbw <= 128) { hipLaunchKernelGGL((k_band_lu_mfma<T, 9, 8>), dim3(nsys), dim3(512 + X), 0, st, a); return true; }
        if (maxbw <= 160) { hipLaunchKernelGGL((k_band_lu_mfma<T, 11, 8>), dim3(nsys), dim3(512 + X), 0, st, a); return true; }
        return false;
    }
    // smallest window W = TP * RB above the half-bandwidth; for W = 160 the
    // variant picks 32 x 32 threads with 5 x 5 blocks (4) or 20 x 20 threads
    // with 8 x 8 blocks (2); 0 = default per precision
    if (maxbw < 80) { hipLaunchKernelGGL((k_band_lu<T, 16, 5>), dim3(nsys), dim3(256), 0, st, a); return true; }
    if (maxbw < 96) { hipLaunchKernelGGL((k_band_lu<T, 16, 6>), dim3(nsys), dim3(256), 0, st, a); return true; }
    if (maxbw < 128) { hipLaunchKernelGGL((k_band_lu<T, 16, 8>), dim3(nsys), dim3(256), 0, st, a); return true; }
    if (maxbw < 160) {
        const bool wide = variant == 4 || (variant == 0 && sizeof(T) == 4);
        if (wide) hipLaunchKernelGGL((k_band_lu<T, 32, 5>), dim3(nsys), dim3(1024), 0, st, a);
        else hipLaunchKernelGGL((k_band_lu<T, 20, 8>), dim3(nsys), dim3(400), 0, st, a);
        return true;
    }
    // wider than the blocked kernels' windows (every variant lands here)
    if (maxbw <= LU_MAX_BW) { hipLaunchKernelGGL((k_band_lu<T, 22, 8>), dim3(nsys), dim3(484), 0, st, a); return true; }
    return false;
}

template <typename T, int D>
bool launch_band_solve_d(const SolveArgs<T> &a, int nsys, int nrhs, int maxbw, int maxn, hipStream_t st) {
    dim3 g(nsys, nrhs);
    const size_t sh = (size_t)(maxn + 2 * solve_pad(solve_nr(maxbw))) * sizeof(T);
    if (sh > 160 * 1024) return false;
    switch (solve_nr(maxbw)) {
    case 2: hipLaunchKernelGGL((k_band_solve<T, 2, D>), g, dim3(SOLVE_THREADS), sh, st, a); break;
    case 3: hipLaunchKernelGGL((k_band_solve<T, 3, D>), g, dim3(SOLVE_THREADS), sh, st, a); break;
    case 4: hipLaunchKernelGGL((k_band_solve<T, 4, D>), g, dim3(SOLVE_THREADS), sh, st, a); break;
    default: return false;
    }
    return true;
}

// depth: columns of factor prefetch (16, 32 or 64)
template <typename T>
bool launch_band_solve(const SolveArgs<T> &a, int nsys, int nrhs, int maxbw, int maxn, int depth, hipStream_t st) {
    // automatic depth: 32 columns in flight for FP32, 16 for FP64 (deeper
    // prefetch measured no faster: the column chain, not the loads, sets the pace)
    if (depth != 16 && depth != 32 && depth != 64) depth = sizeof(T) == 4 ? 32 : 16;
    if constexpr (sizeof(T) == 4) {
        if (depth == 64) return launch_band_solve_d<T, 64>(a, nsys, nrhs, maxbw, maxn, st);
    }
    return depth == 16 ? launch_band_solve_d<T, 16>(a, nsys, nrhs, maxbw, maxn, st)
                       : launch_band_solve_d<T, 32>(a, nsys, nrhs, maxbw, maxn, st);
}

void launch_dense_apply(const DenseArgs &a, int nsys, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_apply, dim3((a.n + 63) / 64, nsys), dim3(1024), 0, st, a);
}

void launch_merge(const MergeArgs &porous, const MergeArgs &conduit, int nsamples, hipStream_t st) {
    long long n = (long long)(2 * porous.N + 1) * (2 * porous.N + 1) + (long long)(porous.N + 1) * (porous.N + 1);
    hipLaunchKernelGGL(k_merge, dim3(grid_for(n, 256), 2, nsamples), dim3(256), 0, st, porous, conduit);
}
void launch_lag_merged(const MergeArgs &porous, const MergeArgs &conduit, int nsamples, hipStream_t st) {
    const int nb = porous.nper > conduit.nper ? porous.nper : conduit.nper;
    hipLaunchKernelGGL(k_lag_merged, dim3(nb, 2, nsamples), dim3(256), 0, st, porous, conduit);
}
void launch_init_corrections(const InitArgs &a, int nsys, hipStream_t st) {
    hipLaunchKernelGGL(k_init_corrections, dim3(nsys), dim3(256), 0, st, a);
}
void launch_dense_newton(const DenseNewtonArgs &a, int nsamples, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_newton, dim3((a.d.n + 63) / 64, nsamples), dim3(1024), 0, st, a);
}
void launch_dense_porous(const DensePorousArgs &a, int nsys, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_porous, dim3((a.d.n + 63) / 64, nsys), dim3(1024), 0, st, a);
}
void launch_newton_start(const NewtonStartArgs &a, int nsamples, hipStream_t st) {
    const long long work = a.band_n > a.nu2 + a.np ? a.band_n : a.nu2 + a.np;
    const int nb = (int)std::min<long long>(1024, (work + 255) / 256);
    hipLaunchKernelGGL(k_newton_start, dim3(nb > 0 ? nb : 1, nsamples), dim3(256), 0, st, a);
}
__global__ void k_time_level(long long *level, long long stride, double dt, double *tf) {
    const long long m = *level;
    *level = m + stride;
    const double t = (double)m * dt;
    const double c = cos(t);
    tf[0] = c;
    tf[1] = sin(t);
    tf[2] = c * c;
}
void launch_time_level(long long *level, long long stride, double dt, double *tf, hipStream_t st) {
    hipLaunchKernelGGL(k_time_level, dim3(1), dim3(1), 0, st, level, stride, dt, tf);
}
__global__ void k_zero_ints(int *p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) p[i] = 0;
}
void launch_zero_ints(int *p, long long n, hipStream_t st) {
    if (n <= 0) return;
    const int nb = (int)std::min<long long>(256, (n + 255) / 256);
    hipLaunchKernelGGL(k_zero_ints, dim3(nb), dim3(256), 0, st, p, n);
}
__global__ void k_zero_fill(uint4 *p, long long n16, unsigned char *tail, int ntail) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}
void launch_zero_fill(void *p, size_t bytes, hipStream_t st) {
    if (bytes == 0) return;
    const long long n16 = (long long)(bytes / 16);
    const int ntail = (int)(bytes % 16);
    const int nb = (int)std::min<long long>(2048, std::max<long long>(1, (n16 + 255) / 256));
    hipLaunchKernelGGL(k_zero_fill, dim3(nb), dim3(256), 0, st, (uint4 *)p, n16, (unsigned char *)p + n16 * 16, ntail);
}
void launch_newton_update(const NewtonArgs &a, int nsamples, hipStream_t st) {
    hipLaunchKernelGGL(k_newton_update, dim3(nsamples), dim3(256), 0, st, a);
}
template void launch_porous_assemble<float>(const AssembleArgs<float> &, int, hipStream_t);
template void launch_porous_assemble<double>(const AssembleArgs<double> &, int, hipStream_t);
template void launch_oseen_assemble<float>(const OseenApplyArgs<float> &, int, int, hipStream_t);
template void launch_oseen_assemble<double>(const OseenApplyArgs<double> &, int, int, hipStream_t);
template void launch_oseen_rows<double>(const OseenApplyArgs<double> &, int, int, int, hipStream_t);
template bool launch_band_lu<float>(const BandArgs<float> &, int, int, int, hipStream_t);
template bool launch_band_lu<double>(const BandArgs<double> &, int, int, int, hipStream_t);
template bool launch_band_solve<float>(const SolveArgs<float> &, int, int, int, int, int, hipStream_t);
template bool launch_band_solve<double>(const SolveArgs<double> &, int, int, int, int, int, hipStream_t);

}  // namespace lp
