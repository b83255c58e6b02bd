// The paper's own discretisation (Section 6: MINI elements in the conduit,
// P1 porous pressures) with Algorithm 1 (partitioned time stepping, Section
// 3.3) on one grid, FP64, on the device.
//
// Per step t_n -> t_{n+1}:
//   1. the three porous P1 systems with the lagged exchange terms and the
//      lagged Gamma flux u^n . n_c (Algorithm 1 Step 1; the matrices are
//      constant and factored once), one node-gather right-hand side kernel and
//      one band solve launch;
//   2. backward-Euler Navier-Stokes on the MINI space with the lagged p_F^n on
//      Gamma (Algorithm 1 Step 2) by chord iterations: one row-gather kernel
//      writes -F (and, at the step's first iterate, the Jacobian band, which
//      the library's band LU factors), the band solve gives the update, and
//      one block applies it and forms the norms of the convergence test.
//
// Unknowns of the Navier-Stokes system, in band order: vertex by vertex (x
// fastest), each vertex (i, j) with i, j < N holding [u_x, u_y, the bubbles
// (u_x, u_y) of its cell's two triangles, p], the others [u_x, u_y, p].  A
// vertex's pressure follows the bubbles of its own cell, and every other
// pressure row meets an eliminated bubble of a neighbouring cell first, so
// the elimination without pivoting takes each pressure pivot from the
// bubbles' Schur complement (negative) and never meets the zero diagonal of
// the saddle point.  Rows gather their own entries over the elements that
// touch their basis function: no atomics, deterministic.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "kernels.h"

namespace lp {
namespace {

__constant__ double c_mw[MINI_NQ];
__constant__ double c_mphi[MINI_NQ][4];
__constant__ double c_mdphi[2][MINI_NQ][4][2];

// The elements (cell ci, cj, orientation t) holding vertex (i, j) and the
// vertex's local index there; T0 = {(0,0),(1,0),(1,1)}, T1 = {(0,0),(1,1),(0,1)}.
__device__ int vertex_elements(int i, int j, int N, int el[6][4]) {
    const int cand[6][4] = {{i, j, 0, 0}, {i, j, 1, 0}, {i - 1, j, 0, 1},
                            {i - 1, j - 1, 0, 2}, {i - 1, j - 1, 1, 1}, {i, j - 1, 1, 2}};
    int n = 0;
    for (int k = 0; k < 6; ++k)
        if (cand[k][0] >= 0 && cand[k][0] < N && cand[k][1] >= 0 && cand[k][1] < N) {
            for (int m = 0; m < 4; ++m) el[n][m] = cand[k][m];
            ++n;
        }
    return n;
}

struct MiniNsArgs {
    int N, bw;
    const int32_t *vu;            // band index of u_x at each conduit vertex (u_y follows)
    const int32_t *vp;            // band index of p at each conduit vertex
    const int32_t *eb;            // band index of each element's bubble u_x (u_y follows)
    const int8_t *dirv;           // conduit vertex on the physical boundary (velocity fixed)
    const double *x;              // Newton iterate (band order)
    const double *xo;             // state at t_n (band order)
    const double *pF0;            // porous p_F at t_n (vertex lattice)
    const double *load[2][3];     // MINI loads of f_c: cos t, sin t, cos^2 t parts
    double ct, st, c2t;           // cos t_{n+1}, sin t_{n+1}, cos^2 t_{n+1}
    double *band;                 // Jacobian, entry (r, c) at c (2 bw + 1) + bw + r - c (cleared)
    double *rhs;                  // -F
    const Coef *co;               // per sample
    int jac;                      // 1: also write the Jacobian rows (0: -F only)
    const int *done;              // per sample: converged this step (rows skipped)
    // sample s (grid y) at x + s nx, band + s nx (2 bw + 1), pF0 + s np, load + s nl
    long long nx, np, nl;
};

__global__ void __launch_bounds__(128) k_mini_ns_rows(MiniNsArgs a) {
    const int N = a.N, n1 = N + 1, nv = n1 * n1, ne = 2 * N * N;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int smp = blockIdx.y;
    if (r >= 3 * nv + 2 * ne || a.done[smp]) return;
    const long long ld = 2 * a.bw + 1;
    // this sample's vectors and band (local pointers: the argument block is
    // left as it is, so that no part of it needs a private copy)
    const double *X = a.x + smp * a.nx, *XO = a.xo + smp * a.nx, *PF0 = a.pF0 + smp * a.np;
    double *RHS = a.rhs + smp * a.nx, *BAND = a.band + smp * a.nx * ld;
    const long long loff = smp * a.nl;
    int kind, c, v = -1, e = -1;
    if (r < 3 * nv) { v = r / 3; kind = r % 3; c = kind; }
    else { e = (r - 3 * nv) / 2; c = (r - 3 * nv) % 2; kind = 3; }
    const int R = kind == 2 ? a.vp[v] : kind < 2 ? a.vu[v] + c : a.eb[e] + c;
    if (kind < 2 && a.dirv[v]) {
        if (a.jac) BAND[(long long)R * ld + a.bw] = 1.0;
        RHS[R] = 0.0;
        return;
    }
    const double h = 1.0 / N, ih = (double)N, h2 = h * h;
    const Coef &co = a.co[smp];
    const double eta = co.eta, mdt = co.eta / co.dt, visc = co.nu * co.eta;
    const double ceta = co.convection ? co.eta : 0.0;          // Stokes: no b_N
    // the elements touching the row's basis function, in a fixed order:
    // for a vertex (i, j) the triangles (cell, orientation, local index)
    // (i,j,0,0) (i,j,1,0) (i-1,j,0,1) (i-1,j-1,0,2) (i-1,j-1,1,1) (i,j-1,1,2),
    // for a bubble its own element (indices computed, no local tables)
    const int vi = kind == 3 ? 0 : v % n1, vj = kind == 3 ? 0 : v / n1;
    auto put = [&](int col, double val) { BAND[(long long)col * ld + a.bw + R - col] += val; };
    double F = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int ci, cj, t;
        const int tv = k <= 1 ? 0 : (k == 2 || k == 4) ? 1 : 2;      // a vertex's local index there
        if (kind == 3) {
            if (k > 0) break;
            const int cell = e >> 1;
            ci = cell % N;
            cj = cell / N;
            t = e & 1;
        } else {
            ci = vi - ((k == 2 || k == 3 || k == 4) ? 1 : 0);
            cj = vj - (k >= 3 ? 1 : 0);
            t = (k == 1 || k == 4 || k == 5) ? 1 : 0;
            if (ci < 0 || ci >= N || cj < 0 || cj >= N) continue;
        }
        int iu[4], ip[3];
        for (int b = 0; b < 3; ++b) {
            const int vb = (ci + off1a(t, b)) + n1 * (cj + off1b(t, b));
            iu[b] = a.vu[vb];
            ip[b] = a.vp[vb];
        }
        iu[3] = a.eb[2 * (ci + N * cj) + t];
        double wv[2][4], wo[2][4], pv[3];
        for (int b = 0; b < 4; ++b)
            for (int d = 0; d < 2; ++d) { wv[d][b] = X[iu[b] + d]; wo[d][b] = XO[iu[b] + d]; }
        for (int b = 0; b < 3; ++b) pv[b] = X[ip[b]];
        double Jv[4][2] = {}, Jp[3] = {};
        for (int q = 0; q < MINI_NQ; ++q) {
            const double wq = c_mw[q] * h2;
            double phi[4], g[4][2];
            for (int b = 0; b < 4; ++b) {
                phi[b] = c_mphi[q][b];
                // both orientations' tables at the wave-uniform point q (scalar
                // loads), then this lane's orientation
                g[b][0] = (t ? c_mdphi[1][q][b][0] : c_mdphi[0][q][b][0]) * ih;
                g[b][1] = (t ? c_mdphi[1][q][b][1] : c_mdphi[0][q][b][1]) * ih;
            }
            double w[2], wold[2], gw[2][2];
            for (int d = 0; d < 2; ++d) {
                w[d] = wold[d] = gw[d][0] = gw[d][1] = 0.0;
                for (int b = 0; b < 4; ++b) {
                    w[d] += wv[d][b] * phi[b];
                    wold[d] += wo[d][b] * phi[b];
                    gw[d][0] += wv[d][b] * g[b][0];
                    gw[d][1] += wv[d][b] * g[b][1];
                }
            }
            const double pq = pv[0] * phi[0] + pv[1] * phi[1] + pv[2] * phi[2];
            // the row's test function and component by selects (no indexing
            // of these small arrays by run-time values)
            const double fa = kind == 3 ? phi[3] : phi[tv];
            const double ga0 = kind == 3 ? g[3][0] : g[tv][0], ga1 = kind == 3 ? g[3][1] : g[tv][1];
            if (kind == 2) {
                // eta int psi_a div u; Jacobian eta int psi_a d_d phi_b
                const double fe = wq * eta * fa;
                F += fe * (gw[0][0] + gw[1][1]);
                for (int b = 0; b < 4; ++b)
                    for (int d = 0; d < 2; ++d) Jv[b][d] += fe * g[b][d];
            } else {
                const double gac = c ? ga1 : ga0;
                const double wc = c ? w[1] : w[0], woc = c ? wold[1] : wold[0];
                const double gwc0 = c ? gw[1][0] : gw[0][0], gwc1 = c ? gw[1][1] : gw[0][1];   // d_0 u_c, d_1 u_c
                const double gw0c = c ? gw[0][1] : gw[0][0], gw1c = c ? gw[1][1] : gw[1][0];   // d_c u_0, d_c u_1
                // (eta/dt)(u - u^n) + 2 nu eta D(u) : D(v) + eta (u.grad)u . v - eta p div v
                F += wq * (mdt * (wc - woc) * fa + visc * (ga0 * (gwc0 + gw0c) + ga1 * (gwc1 + gw1c)) +
                           ceta * (w[0] * gwc0 + w[1] * gwc1) * fa - eta * pq * gac);
                for (int b = 0; b < 4; ++b) {
                    const double wgb = w[0] * g[b][0] + w[1] * g[b][1];
                    const double diag = mdt * fa * phi[b] + visc * (ga0 * g[b][0] + ga1 * g[b][1]) + ceta * wgb * fa;
                    const double gbc = c ? g[b][1] : g[b][0];
                    for (int d = 0; d < 2; ++d) {
                        const double ga_d = d == 0 ? ga0 : ga1;
                        const double gwcd = d == 0 ? gwc0 : gwc1;
                        Jv[b][d] += wq * ((c == d ? diag : 0.0) + visc * ga_d * gbc + ceta * phi[b] * gwcd * fa);
                    }
                }
                for (int b = 0; b < 3; ++b) Jp[b] -= wq * eta * phi[b] * gac;
            }
        }
        if (a.jac) {
            for (int b = 0; b < 4; ++b)
                for (int d = 0; d < 2; ++d) put(iu[b] + d, Jv[b][d]);
            if (kind != 2)
                for (int b = 0; b < 3; ++b) put(ip[b], Jp[b]);
        }
    }
    if (kind != 2) {
        // sources (time-separable loads)
        const int pub = kind == 3 ? nv + e : v;
        const double *L0 = c ? a.load[1][0] : a.load[0][0], *L1 = c ? a.load[1][1] : a.load[0][1];
        const double *L2 = c ? a.load[1][2] : a.load[0][2];
        F -= eta * (L0[loff + pub] * a.ct + L1[loff + pub] * a.st + L2[loff + pub] * a.c2t);
        // Gamma (conduit row j = 0, n_c = (0, -1)): Beavers-Joseph eta beta int u_x v_x,
        // + c_tau int d_x p_F v_x and -(eta/rho) int p_F v_y with the lagged p_F^n
        if (kind < 2 && v / n1 == 0) {
            const int i = v % n1;
            for (int s = -1; s <= 0; ++s) {
                const int i0 = i + s;                       // edge [i0, i0 + 1]
                if (i0 < 0 || i0 >= N) continue;
                const int la = i - i0;                      // the row's end of the edge
                for (int lb = 0; lb < 2; ++lb) {
                    const int ib = i0 + lb;
                    const double G = h * (la == lb ? 1.0 / 3.0 : 1.0 / 6.0);
                    const double Gx = lb == 0 ? -0.5 : 0.5;
                    const double pF = PF0[ib + n1 * N];
                    if (c == 0) {
                        const int col = a.vu[ib];
                        if (a.jac) put(col, eta * co.beta * G);
                        F += eta * co.beta * G * X[col] + co.ctau * Gx * pF;
                    } else {
                        F -= eta / co.rho * G * pF;
                    }
                }
            }
        }
    }
    RHS[R] = -F;
}

// Velocity at t_{n+1} on the physical boundary (Newton start: the state of
// t_n elsewhere)
__global__ void k_mini_dirichlet(int N, const int32_t *vu, const int8_t *dirv, const double *ex_u1,
                                 const double *ex_u2, double ct, double *x, long long nx) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (N + 1) * (N + 1) || !dirv[v]) return;
    x += blockIdx.y * nx;
    x[vu[v]] = ex_u1[v] * ct;
    x[vu[v] + 1] = ex_u2[v] * ct;
}

// per sample (block): unless it has converged, x += d over its Navier-Stokes
// unknowns, then the test ||d|| <= 1e-13 ||x|| (relative update) marks it done
__global__ void __launch_bounds__(1024) k_mini_update(int n, const double *d, double *x, int *done) {
    __shared__ double sd[1024], sx[1024];
    const int smp = blockIdx.x;
    if (done[smp]) return;
    d += (long long)smp * n;
    x += (long long)smp * n;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double di = d[i], xi = x[i] + di;
        x[i] = xi;
        a += di * di;
        b += xi * xi;
    }
    sd[threadIdx.x] = a;
    sx[threadIdx.x] = b;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sd[threadIdx.x] += sd[threadIdx.x + s];
            sx[threadIdx.x] += sx[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && sd[0] <= 1e-26 * sx[0]) done[smp] = 1;
}

struct MiniPorArgs {
    int N, bw;
    const double *P;              // p_F, p_f, p_m at t_n (3 (N+1)^2, vertex lattice)
    const double *xo;             // conduit state at t_n (band order): u_y on Gamma
    const int32_t *vu;            // conduit band index of u_x per vertex
    const double *ex[3];          // spatial parts of the exact p_F, p_f, p_m
    const double *load[3][2];     // P1 loads: cos t, sin t parts
    double ct, st;
    double *band;                 // three band matrices (setup), n (2 bw + 1) each
    double *rhs;                  // three right-hand sides (per step)
    const Coef *co;               // per sample
    // sample s (grid y) at P, rhs + s np; band + s np (2 bw + 1); xo + s nx; load + s nv
    long long np, nx;
};

// Porous row of vertex v: mode 0 writes the three band rows (setup), mode 1
// the three right-hand sides of the step
template <int MODE>
__global__ void __launch_bounds__(128) k_mini_porous(MiniPorArgs a) {
    const int N = a.N, n1 = N + 1, nv = n1 * n1;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int smp = blockIdx.y;
    const long long ld = 2 * a.bw + 1, bs = (long long)nv * ld;
    if (MODE == 0) a.band += smp * a.np * ld;
    else {
        a.P += smp * a.np;
        a.rhs += smp * a.np;
        a.xo += smp * a.nx;
    }
    const long long loff = (long long)smp * nv;
    const int i = v % n1, j = v / n1;
    const bool dir = i == 0 || i == N || j == 0;
    const Coef &co = a.co[smp];
    if (dir) {
        if (MODE == 0) for (int f = 0; f < 3; ++f) a.band[f * bs + (long long)v * ld + a.bw] = 1.0;
        else for (int f = 0; f < 3; ++f) a.rhs[f * nv + v] = a.ex[f][v] * a.ct;
        return;
    }
    const double h = 1.0 / N, ih = (double)N, h2 = h * h;
    const double cm[3] = {co.tau[0] + co.sst, co.tau[1] + co.s + co.sst, co.tau[2] + co.s};
    int el[6][4];
    const int nel = vertex_elements(i, j, N, el);
    double m[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < nel; ++k) {
        const int ci = el[k][0], cj = el[k][1], t = el[k][2], ta = el[k][3];
        int vb[3];
        for (int b = 0; b < 3; ++b) vb[b] = (ci + off1a(t, b)) + n1 * (cj + off1b(t, b));
        double Me[3] = {}, Ke[3] = {};
        for (int q = 0; q < MINI_NQ; ++q) {
            const double wq = c_mw[q] * h2;
            for (int b = 0; b < 3; ++b) {
                Me[b] += wq * c_mphi[q][ta] * c_mphi[q][b];
                Ke[b] += wq * ih * ih * (c_mdphi[t][q][ta][0] * c_mdphi[t][q][b][0] + c_mdphi[t][q][ta][1] * c_mdphi[t][q][b][1]);
            }
        }
        if (MODE == 0) {
            for (int f = 0; f < 3; ++f)
                for (int b = 0; b < 3; ++b)
                    a.band[f * bs + (long long)vb[b] * ld + a.bw + v - vb[b]] += cm[f] * Me[b] + co.kap[f] * Ke[b];
        } else {
            for (int f = 0; f < 3; ++f)
                for (int b = 0; b < 3; ++b) m[f] += Me[b] * a.P[f * nv + vb[b]];
        }
    }
    if (MODE == 0) return;
    double gam = 0.0;
    if (j == N) {
        // the lagged flux: + int v_F u^n . n_c = - int v_F u_y^n on Gamma
        for (int s = -1; s <= 0; ++s) {
            const int i0 = i + s;
            if (i0 < 0 || i0 >= N) continue;
            for (int lb = 0; lb < 2; ++lb) {
                const int ib = i0 + lb;
                gam -= h * (i - i0 == lb ? 1.0 / 3.0 : 1.0 / 6.0) * a.xo[a.vu[ib] + 1];
            }
        }
    }
    double Q[3];
    for (int f = 0; f < 3; ++f) Q[f] = a.load[f][0][loff + v] * a.ct + a.load[f][1][loff + v] * a.st;
    a.rhs[v] = Q[0] + co.tau[0] * m[0] + co.sst * m[1] + gam;
    a.rhs[nv + v] = Q[1] + co.tau[1] * m[1] + co.s * m[2] + co.sst * m[0];
    a.rhs[2 * nv + v] = Q[2] + co.tau[2] * m[2] + co.s * m[1];
}

}  // namespace
}  // namespace lp

using lp::Coef;

struct lp_mini {
    int device = 0;
    int problem = LP_MMS_EX1_2D;
    int N = 0, n1 = 0, nv = 0, ne = 0, ns = 1;
    int nns = 0, bw_ns = 0, bw_p = 0, var_ns = 0, var_p = 0;
    std::vector<lp_params> prm;
    double dt = 0.0;
    hipStream_t st = nullptr;
    std::vector<int32_t> vu, vp, eb;
    int32_t steps = 0, its_max = 0, flags = 0;
    double lu_ms = 0.0;           // HIP-event time of the Navier-Stokes factorisations
    int64_t lu_launches = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<void *> bufs;
    // device; per-sample blocks follow each other (stride nns, 3 nv, ...)
    int32_t *d_vu = nullptr, *d_vp = nullptr, *d_eb = nullptr;
    int8_t *d_dirv = nullptr;
    Coef *d_co = nullptr;
    int *d_done = nullptr;
    double *x = nullptr, *xo = nullptr, *d = nullptr, *rhs = nullptr, *band = nullptr;
    double *P = nullptr, *Pn = nullptr, *prhs = nullptr, *pband = nullptr;
    double *ex[8] = {};
    double *ld_p[3][2] = {}, *ld_u[2][3] = {};
    double *fac = nullptr, *pfac = nullptr, *dummy = nullptr, *consts = nullptr;
    int *lflags = nullptr;
    float *lstat = nullptr;
    lp::BandSys *sys_ns = nullptr, *sys_p = nullptr;

    template <typename T>
    bool alloc(T **p, size_t n) {
        void *v = nullptr;
        if (hipMalloc(&v, (n ? n : 1) * sizeof(T)) != hipSuccess) return false;
        bufs.push_back(v);
        *p = (T *)v;
        return true;
    }
    ~lp_mini() {
        for (void *v : bufs) (void)hipFree(v);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (st) (void)hipStreamDestroy(st);
    }
};

namespace {

#define MCHK(expr)                                                                                  \
    do {                                                                                            \
        hipError_t _e = (expr);                                                                     \
        if (_e != hipSuccess)                                                                       \
            return lp::set_error(LP_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

int grid(long long n, int b) { return (int)((n + b - 1) / b); }

Coef coefficients(const lp_params &p, int problem) {
    Coef co{};
    const double mu = p.mu_tilde;
    for (int i = 0; i < 3; ++i) {
        co.tau[i] = p.phi[i] * p.C[i] / p.dt;
        co.kap[i] = p.k[i] / mu;
    }
    co.sst = p.sigma_star * p.k[1] / mu;
    co.s = p.sigma * p.k[2] / mu;
    co.eta = p.eta;
    co.nu = p.nu;
    co.rho = p.rho;
    co.dt = p.dt;
    co.beta = p.alpha * p.nu / std::sqrt(p.k[0]);
    co.ctau = p.eta * p.nu * p.alpha * std::sqrt(p.k[0]) / mu;
    co.convection = problem == LP_EX3_2D ? 0 : 1;               // Example 3's conduit is Stokes
    return co;
}

lp_status mini_init(lp_mini *c) {
    const int N = c->N, n1 = c->n1, nv = c->nv, ne = c->ne, ns = c->ns;
    // band numbering of the Navier-Stokes unknowns
    c->vu.assign(nv, 0);
    c->vp.assign(nv, 0);
    c->eb.assign(ne, 0);
    int pos = 0;
    for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
            const int v = i + n1 * j;
            c->vu[v] = pos;
            pos += 2;
            if (i < N && j < N) {
                c->eb[2 * (i + N * j)] = pos;
                c->eb[2 * (i + N * j) + 1] = pos + 2;
                pos += 4;
            }
            c->vp[v] = pos++;
        }
    c->nns = pos;
    int bw = 0;
    for (int cj = 0; cj < N; ++cj)
        for (int ci = 0; ci < N; ++ci)
            for (int t = 0; t < 2; ++t) {
                int lo = c->eb[2 * (ci + N * cj) + t], hi = lo + 1;
                for (int b = 0; b < 3; ++b) {
                    const int vb = (ci + lp::off1a(t, b)) + n1 * (cj + lp::off1b(t, b));
                    lo = std::min(lo, std::min(c->vu[vb], c->vp[vb]));
                    hi = std::max(hi, std::max(c->vu[vb] + 1, c->vp[vb]));
                }
                bw = std::max(bw, hi - lo);
            }
    c->bw_ns = bw;
    c->bw_p = N + 2;
    c->var_ns = bw <= 160 ? 9 : 0;
    c->var_p = c->bw_p <= 160 ? 9 : 0;
    if (bw > lp::LU_MAX_BW || lp::solve_nr(bw) == 0)
        return lp::set_error(LP_ERR_UNSUPPORTED, "the MINI Navier-Stokes half-bandwidth " + std::to_string(bw) +
                                                     " exceeds the band kernels' window of " +
                                                     std::to_string(lp::LU_MAX_BW));
    // conduit velocity fixed on the physical boundary: every side but Gamma
    // for Example 1; for the Example-3-type variant only the cased side walls
    // (their end points included), the rest of the top being the outflow
    const bool ex3 = c->problem == LP_EX3_2D;
    std::vector<int8_t> dirv(nv);
    for (int v = 0; v < nv; ++v) {
        const int i = v % n1, j = v / n1;
        dirv[v] = i == 0 || i == N || (!ex3 && j == N);
    }
    // reference data, loads (per sample: they depend on the parameters), exact spatial parts
    lp::MiniRef ref;
    lp::build_mini_refdata(ref);
    MCHK(hipMemcpyToSymbol(HIP_SYMBOL(lp::c_mw), ref.w, sizeof(ref.w)));
    MCHK(hipMemcpyToSymbol(HIP_SYMBOL(lp::c_mphi), ref.phi, sizeof(ref.phi)));
    MCHK(hipMemcpyToSymbol(HIP_SYMBOL(lp::c_mdphi), ref.dphi, sizeof(ref.dphi)));
    std::vector<double> loads[5][3], ex[8];
    for (int f = 0; f < 5; ++f)
        for (int k = 0; k < 3; ++k) loads[f][k].assign((size_t)ns * (f < 3 ? nv : nv + ne), 0.0);
    if (ex3) {
        // no sources; fixed porous pressures on Gamma_in (and as the initial
        // state), a conduit at rest
        const double pin[3] = {1.0e3, 1.6e3, 4.0e3};
        for (int f = 0; f < 3; ++f) ex[f].assign(nv, pin[f]);
        for (int f = 3; f < 6; ++f) ex[f].assign(nv, 0.0);
        for (int f = 6; f < 8; ++f) ex[f].assign(ne, 0.0);
    } else {
        for (int smp = 0; smp < ns; ++smp) {
            std::vector<double> one[5][3];
            lp::mini_source_loads(N, c->prm[smp], one);
            for (int f = 0; f < 5; ++f)
                for (int k = 0; k < 3; ++k)
                    std::copy(one[f][k].begin(), one[f][k].end(), loads[f][k].begin() + (size_t)smp * one[f][k].size());
        }
        lp::mini_exact_spatial(N, ex);
    }
    std::vector<Coef> co(ns);
    for (int smp = 0; smp < ns; ++smp) co[smp] = coefficients(c->prm[smp], c->problem);
    // device buffers
    const long long nns = c->nns;
    const long long ldn = 2LL * c->bw_ns + 1, ldp = 2LL * c->bw_p + 1;
    const int ldf_ns = 64 * lp::solve_nr(c->bw_ns), ldf_p = 64 * lp::solve_nr(c->bw_p);
    const long long fac_ns = 2LL * nns * ldf_ns + nns, fac_p = 2LL * nv * ldf_p + nv;
    if (!c->alloc(&c->d_vu, nv) || !c->alloc(&c->d_vp, nv) || !c->alloc(&c->d_eb, ne) || !c->alloc(&c->d_dirv, nv) ||
        !c->alloc(&c->d_co, ns) || !c->alloc(&c->d_done, ns) || !c->alloc(&c->x, ns * nns) ||
        !c->alloc(&c->xo, ns * nns) || !c->alloc(&c->d, ns * nns) || !c->alloc(&c->rhs, ns * nns) ||
        !c->alloc(&c->band, ns * nns * ldn) || !c->alloc(&c->P, 3LL * ns * nv) || !c->alloc(&c->Pn, 3LL * ns * nv) ||
        !c->alloc(&c->prhs, 3LL * ns * nv) || !c->alloc(&c->pband, 3LL * ns * nv * ldp) ||
        !c->alloc(&c->fac, ns * fac_ns) || !c->alloc(&c->pfac, 3LL * ns * fac_p) ||
        !c->alloc(&c->dummy, 3LL * ns * lp::LU_DUMMY_PER_SYS) || !c->alloc(&c->consts, 2) ||
        !c->alloc(&c->lflags, 1) || !c->alloc(&c->lstat, 2) || !c->alloc(&c->sys_ns, ns) || !c->alloc(&c->sys_p, 3LL * ns))
        return lp::set_error(LP_ERR_ALLOC, "device allocation failed");
    for (int f = 0; f < 8; ++f)
        if (!c->alloc(&c->ex[f], ex[f].size())) return lp::set_error(LP_ERR_ALLOC, "device allocation failed");
    for (int f = 0; f < 3; ++f)
        for (int k = 0; k < 2; ++k)
            if (!c->alloc(&c->ld_p[f][k], loads[f][k].size())) return lp::set_error(LP_ERR_ALLOC, "device allocation failed");
    for (int cc = 0; cc < 2; ++cc)
        for (int k = 0; k < 3; ++k)
            if (!c->alloc(&c->ld_u[cc][k], loads[3 + cc][k].size()))
                return lp::set_error(LP_ERR_ALLOC, "device allocation failed");
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    MCHK(up(c->d_vu, c->vu.data(), nv * sizeof(int32_t)));
    MCHK(up(c->d_vp, c->vp.data(), nv * sizeof(int32_t)));
    MCHK(up(c->d_eb, c->eb.data(), ne * sizeof(int32_t)));
    MCHK(up(c->d_dirv, dirv.data(), nv));
    MCHK(up(c->d_co, co.data(), ns * sizeof(Coef)));
    for (int f = 0; f < 8; ++f) MCHK(up(c->ex[f], ex[f].data(), ex[f].size() * sizeof(double)));
    for (int f = 0; f < 3; ++f)
        for (int k = 0; k < 2; ++k) MCHK(up(c->ld_p[f][k], loads[f][k].data(), loads[f][k].size() * sizeof(double)));
    for (int cc = 0; cc < 2; ++cc)
        for (int k = 0; k < 3; ++k)
            MCHK(up(c->ld_u[cc][k], loads[3 + cc][k].data(), loads[3 + cc][k].size() * sizeof(double)));
    // initial data (t = 0): vertex values, bubbles exact at the centroids; the
    // same for every sample (the exact fields do not depend on the parameters)
    std::vector<double> x0(nns, 0.0), P0(3 * (size_t)nv);
    for (int v = 0; v < nv; ++v) {
        x0[c->vu[v]] = ex[3][v];
        x0[c->vu[v] + 1] = ex[4][v];
        x0[c->vp[v]] = ex[5][v];
        for (int f = 0; f < 3; ++f) P0[f * (size_t)nv + v] = ex[f][v];
    }
    for (int cj = 0; cj < N; ++cj)
        for (int ci = 0; ci < N; ++ci)
            for (int t = 0; t < 2; ++t) {
                const int e = 2 * (ci + N * cj) + t;
                for (int cc = 0; cc < 2; ++cc) {
                    double mean = 0.0;
                    for (int b = 0; b < 3; ++b) mean += ex[3 + cc][(ci + lp::off1a(t, b)) + n1 * (cj + lp::off1b(t, b))];
                    x0[c->eb[e] + cc] = ex[6 + cc][e] - mean / 3.0;
                }
            }
    for (int smp = 0; smp < ns; ++smp) {
        MCHK(up(c->x + smp * nns, x0.data(), nns * sizeof(double)));
        MCHK(up(c->P + 3LL * smp * nv, P0.data(), P0.size() * sizeof(double)));
    }
    const double consts[2] = {0.0, 1.0};
    MCHK(up(c->consts, consts, sizeof(consts)));
    std::vector<lp::BandSys> sns(ns), sp(3 * (size_t)ns);
    for (int smp = 0; smp < ns; ++smp) {
        sns[smp] = lp::BandSys{smp * nns * ldn, 0, smp * nns, smp * fac_ns, 0, (int)nns, c->bw_ns, 1, ldf_ns};
        for (int f = 0; f < 3; ++f) {
            const long long k = 3LL * smp + f;
            sp[k] = lp::BandSys{k * nv * ldp, 0, k * nv, k * fac_p, 0, nv, c->bw_p, 1, ldf_p};
        }
    }
    MCHK(up(c->sys_ns, sns.data(), sns.size() * sizeof(lp::BandSys)));
    MCHK(up(c->sys_p, sp.data(), sp.size() * sizeof(lp::BandSys)));
    MCHK(hipMemset(c->fac, 0, ns * fac_ns * sizeof(double)));
    MCHK(hipMemset(c->pfac, 0, 3LL * ns * fac_p * sizeof(double)));
    MCHK(hipMemset(c->pband, 0, 3LL * ns * nv * ldp * sizeof(double)));
    MCHK(hipMemset(c->lflags, 0, sizeof(int)));
    MCHK(hipMemset(c->lstat, 0, 2 * sizeof(float)));
    // the constant porous matrices, factored once
    lp::MiniPorArgs pa{};
    pa.N = N;
    pa.bw = c->bw_p;
    pa.band = c->pband;
    pa.co = c->d_co;
    pa.np = 3LL * nv;
    pa.nx = nns;
    hipLaunchKernelGGL((lp::k_mini_porous<0>), dim3(grid(nv, 128), ns), dim3(128), 0, c->st, pa);
    lp::BandArgs<double> ba{c->sys_p, c->pband, c->pfac, c->lflags, nullptr, c->dummy, c->consts, c->consts + 1, c->lstat};
    if (!lp::launch_band_lu<double>(ba, 3 * ns, c->bw_p, c->var_p, c->st))
        return lp::set_error(LP_ERR_UNSUPPORTED, "porous factorisation window");
    MCHK(hipGetLastError());
    MCHK(hipStreamSynchronize(c->st));
    return LP_OK;
}

lp_status mini_step(lp_mini *c) {
    const int N = c->N, nv = c->nv, ns = c->ns;
    const long long nns = c->nns;
    const double t1 = (double)(c->steps + 1) * c->dt;
    // Example 1's data are a(x) cos t (sources also sin t, cos^2 t); the
    // Example-3-type variant's boundary data are constant in time
    const bool ex3 = c->problem == LP_EX3_2D;
    const double ct = ex3 ? 1.0 : std::cos(t1), st = ex3 ? 0.0 : std::sin(t1);
    // Step 1: porous pressures at t_{n+1}, every sample
    lp::MiniPorArgs pa{};
    pa.N = N;
    pa.bw = c->bw_p;
    pa.P = c->P;
    pa.xo = c->x;
    pa.vu = c->d_vu;
    for (int f = 0; f < 3; ++f) {
        pa.ex[f] = c->ex[f];
        for (int k = 0; k < 2; ++k) pa.load[f][k] = c->ld_p[f][k];
    }
    pa.ct = ct;
    pa.st = st;
    pa.rhs = c->prhs;
    pa.co = c->d_co;
    pa.np = 3LL * nv;
    pa.nx = nns;
    hipLaunchKernelGGL((lp::k_mini_porous<1>), dim3(grid(nv, 128), ns), dim3(128), 0, c->st, pa);
    lp::SolveArgs<double> sp{c->sys_p, c->pfac, c->prhs, c->Pn, nullptr, 1, nullptr, c->consts, c->consts + 1, c->consts};
    sp.assign = 1;
    if (!lp::launch_band_solve<double>(sp, 3 * ns, 1, c->bw_p, nv, 0, c->st))
        return lp::set_error(LP_ERR_UNSUPPORTED, "porous band solve size");
    // Step 2: Navier-Stokes at t_{n+1} from (u^n, p^n), every sample
    MCHK(hipMemcpyAsync(c->xo, c->x, ns * nns * sizeof(double), hipMemcpyDeviceToDevice, c->st));
    MCHK(hipMemsetAsync(c->d_done, 0, ns * sizeof(int), c->st));
    hipLaunchKernelGGL(lp::k_mini_dirichlet, dim3(grid(nv, 128), ns), dim3(128), 0, c->st, N, c->d_vu, c->d_dirv,
                       c->ex[3], c->ex[4], ct, c->x, nns);
    lp::MiniNsArgs na{};
    na.N = N;
    na.bw = c->bw_ns;
    na.vu = c->d_vu;
    na.vp = c->d_vp;
    na.eb = c->d_eb;
    na.dirv = c->d_dirv;
    na.x = c->x;
    na.xo = c->xo;
    na.pF0 = c->P;
    for (int cc = 0; cc < 2; ++cc)
        for (int k = 0; k < 3; ++k) na.load[cc][k] = c->ld_u[cc][k];
    na.ct = ct;
    na.st = st;
    na.c2t = ct * ct;
    na.band = c->band;
    na.rhs = c->rhs;
    na.co = c->d_co;
    na.done = c->d_done;
    na.nx = nns;
    na.np = 3LL * nv;
    na.nl = (long long)nv + c->ne;
    const long long nband = ns * nns * (2LL * c->bw_ns + 1);
    const int nrows = 3 * nv + 2 * c->ne;
    lp::BandArgs<double> ba{c->sys_ns, c->band, c->fac, c->lflags, nullptr, c->dummy, c->consts, c->consts + 1, c->lstat};
    lp::SolveArgs<double> sa{c->sys_ns, c->fac, c->rhs, c->d, nullptr, 1, nullptr, c->consts, c->consts + 1, c->consts};
    sa.assign = 1;
    // chord iterations: the Jacobian is formed and factored at the first
    // iterate of the step and applied to the exact residual of every iterate,
    // so the step reaches the same fixed point at the same tolerance; a sample
    // that has converged keeps its iterate while the others go on
    const int maxit = 30;
    int it = 0;
    bool conv = false;
    std::vector<int> done(ns);
    while (it < maxit && !conv) {
        ++it;
        na.jac = it == 1;
        if (na.jac) MCHK(hipMemsetAsync(c->band, 0, nband * sizeof(double), c->st));
        hipLaunchKernelGGL(lp::k_mini_ns_rows, dim3(grid(nrows, 128), ns), dim3(128), 0, c->st, na);
        if (na.jac) {
            MCHK(hipEventRecord(c->ev[0], c->st));
            if (!lp::launch_band_lu<double>(ba, ns, c->bw_ns, c->var_ns, c->st))
                return lp::set_error(LP_ERR_UNSUPPORTED, "Navier-Stokes factorisation window");
            MCHK(hipEventRecord(c->ev[1], c->st));
        }
        if (!lp::launch_band_solve<double>(sa, ns, 1, c->bw_ns, (int)nns, 0, c->st))
            return lp::set_error(LP_ERR_UNSUPPORTED, "Navier-Stokes band solve size");
        hipLaunchKernelGGL(lp::k_mini_update, dim3(ns), dim3(1024), 0, c->st, (int)nns, c->d, c->x, c->d_done);
        MCHK(hipMemcpyAsync(done.data(), c->d_done, ns * sizeof(int), hipMemcpyDeviceToHost, c->st));
        MCHK(hipStreamSynchronize(c->st));
        conv = std::all_of(done.begin(), done.end(), [](int v) { return v != 0; });
        if (na.jac) {
            float ms = 0.f;
            MCHK(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
            c->lu_ms += ms;
            c->lu_launches += 1;
        }
    }
    MCHK(hipGetLastError());
    std::swap(c->P, c->Pn);
    c->steps += 1;
    c->its_max = std::max(c->its_max, it);
    if (!conv) c->flags |= 2;
    return LP_OK;
}

}  // namespace

extern "C" {

lp_status lp_mini_setup(int32_t n, int32_t problem, const lp_params *samples, int32_t nsamples, int32_t device,
                        lp_mini **out) {
    if (!out || !samples) return lp::set_error(LP_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (problem != LP_MMS_EX1_2D && problem != LP_EX3_2D)
        return lp::set_error(LP_ERR_ARG, "problem must be LP_MMS_EX1_2D or LP_EX3_2D");
    // with n = 1 every conduit vertex carries Dirichlet velocity: only the
    // bubbles test the pressure, which then keeps an undetermined constant
    if (n < 2) return lp::set_error(LP_ERR_ARG, "n must be >= 2");
    if (nsamples < 1) return lp::set_error(LP_ERR_ARG, "nsamples must be >= 1");
    for (int smp = 0; smp < nsamples; ++smp) {
        const lp_params &p = samples[smp];
        if (!(p.dt > 0.0)) return lp::set_error(LP_ERR_ARG, "dt must be > 0 (sample " + std::to_string(smp) + ")");
        if (p.dt != samples[0].dt)
            return lp::set_error(LP_ERR_ARG, "samples share one dt (sample " + std::to_string(smp) + ")");
        if (!(p.k[0] > 0.0) || !(p.mu_tilde > 0.0) || !(p.rho > 0.0))
            return lp::set_error(LP_ERR_ARG, "k_F, mu_tilde and rho must be > 0 (sample " + std::to_string(smp) + ")");
    }
    int ndev = 0;
    MCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return lp::set_error(LP_ERR_DEVICE, "device id out of range");
    MCHK(hipSetDevice(device));
    lp_mini *c = new lp_mini();
    c->device = device;
    c->problem = problem;
    c->N = n;
    c->n1 = n + 1;
    c->nv = c->n1 * c->n1;
    c->ne = 2 * n * n;
    c->ns = nsamples;
    c->prm.assign(samples, samples + nsamples);
    c->dt = samples[0].dt;
    if (hipStreamCreate(&c->st) != hipSuccess || hipEventCreate(&c->ev[0]) != hipSuccess ||
        hipEventCreate(&c->ev[1]) != hipSuccess) {
        delete c;
        return lp::set_error(LP_ERR_DEVICE, "stream or event creation failed");
    }
    const lp_status s = mini_init(c);
    if (s != LP_OK) {
        delete c;
        return s;
    }
    *out = c;
    return LP_OK;
}

lp_status lp_mini_step(lp_mini *c, int32_t nsteps) {
    if (!c) return lp::set_error(LP_ERR_ARG, "NULL context");
    if (nsteps < 0) return lp::set_error(LP_ERR_ARG, "nsteps must be >= 0");
    MCHK(hipSetDevice(c->device));
    for (int k = 0; k < nsteps; ++k) {
        const lp_status s = mini_step(c);
        if (s != LP_OK) return s;
    }
    int fl = 0;
    MCHK(hipMemcpy(&fl, c->lflags, sizeof(int), hipMemcpyDeviceToHost));
    c->flags |= fl & 4;
    if (c->flags) return lp::set_error(LP_ERR_NOCONV, "a Newton solve reached its cap or a pivot was flagged");
    return LP_OK;
}

lp_status lp_mini_get(lp_mini *c, int32_t sample, int32_t field, double *out, int64_t len, int64_t *needed) {
    if (!c) return lp::set_error(LP_ERR_ARG, "NULL context");
    if (sample < 0 || sample >= c->ns) return lp::set_error(LP_ERR_ARG, "sample out of range");
    const int nv = c->nv, ne = c->ne;
    int64_t need;
    if (field == LP_PF || field == LP_PFMI || field == LP_PM || field == LP_P) need = nv;
    else if (field == LP_U) need = 2LL * (nv + ne);
    else return lp::set_error(LP_ERR_ARG, "unknown field");
    if (needed) *needed = need;
    if (!out) return LP_OK;
    if (len < need) return lp::set_error(LP_ERR_ARG, "output buffer too short");
    MCHK(hipSetDevice(c->device));
    MCHK(hipStreamSynchronize(c->st));
    if (field == LP_PF || field == LP_PFMI || field == LP_PM) {
        const int f = field == LP_PF ? 0 : field == LP_PFMI ? 1 : 2;
        MCHK(hipMemcpy(out, c->P + (3LL * sample + f) * nv, nv * sizeof(double), hipMemcpyDeviceToHost));
        return LP_OK;
    }
    std::vector<double> x(c->nns);
    MCHK(hipMemcpy(x.data(), c->x + (long long)sample * c->nns, x.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (field == LP_P) {
        for (int v = 0; v < nv; ++v) out[v] = x[c->vp[v]];
        return LP_OK;
    }
    const int64_t nb = nv + ne;
    for (int cc = 0; cc < 2; ++cc) {
        for (int v = 0; v < nv; ++v) out[cc * nb + v] = x[c->vu[v] + cc];
        for (int e = 0; e < ne; ++e) out[cc * nb + nv + e] = x[c->eb[e] + cc];
    }
    return LP_OK;
}

lp_status lp_mini_stats(lp_mini *c, int32_t *steps, int32_t *newton_its_max, int32_t *flags, double *lu_ms,
                        int64_t *lu_launches) {
    if (!c) return lp::set_error(LP_ERR_ARG, "NULL context");
    if (lu_ms) *lu_ms = c->lu_ms;
    if (lu_launches) *lu_launches = c->lu_launches;
    if (steps) *steps = c->steps;
    if (newton_its_max) *newton_its_max = c->its_max;
    if (flags) *flags = c->flags;
    return LP_OK;
}

void lp_mini_destroy(lp_mini *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->st);
    delete c;
}

}  // extern "C"
