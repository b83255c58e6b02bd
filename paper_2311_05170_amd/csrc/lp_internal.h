// Internal definitions shared by the host planner, the HIP kernels and the
// C-ABI layer of liblp.  Everything here describes the 2D right-triangle
// lattice discretisation of the paper's model (Section 3.2: P2 velocity and
// porous pressures, P1 conduit pressure) and the per-system tables the
// kernels index.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "lp.h"

namespace lp {

constexpr int NQ = 16;       // kernel quadrature points per triangle (degree 6 exact)
constexpr int POROUS = 0;
constexpr int CONDUIT = 1;
constexpr int KIND_POROUS = 0;
constexpr int KIND_OSEEN = 1;

// P2 node offsets of the two triangle orientations inside a cell, in half-cell
// units: vertices 0,1,2 then midpoints of edges (0,1), (1,2), (0,2).
//   T0 = {(0,0),(1,0),(1,1)}, T1 = {(0,0),(1,1),(0,1)} (cell units).
__host__ __device__ constexpr int off2a(int t, int k) {
    return t == 0 ? (k == 0 ? 0 : k == 1 ? 2 : k == 2 ? 2 : k == 3 ? 1 : k == 4 ? 2 : 1)
                  : (k == 0 ? 0 : k == 1 ? 2 : k == 2 ? 0 : k == 3 ? 1 : k == 4 ? 1 : 0);
}
__host__ __device__ constexpr int off2b(int t, int k) {
    return t == 0 ? (k == 0 ? 0 : k == 1 ? 0 : k == 2 ? 2 : k == 3 ? 0 : k == 4 ? 1 : 1)
                  : (k == 0 ? 0 : k == 1 ? 2 : k == 2 ? 2 : k == 3 ? 1 : k == 4 ? 2 : 1);
}
// P1 vertex offsets (cell units)
__host__ __device__ constexpr int off1a(int t, int k) { return t == 0 ? (k == 0 ? 0 : 1) : (k == 1 ? 1 : 0); }
__host__ __device__ constexpr int off1b(int t, int k) { return t == 0 ? (k == 2 ? 1 : 0) : (k == 0 ? 0 : 1); }

// Reference data for a cell of unit size (h = 1); kernels rescale by h.
struct RefData {
    double phi[NQ][6];          // P2 values at the quadrature points (same for both orientations)
    double dphi[2][NQ][6][2];   // P2 gradients (unit cell) per orientation
    double psi[NQ][3];          // P1 values
    double w[NQ];               // weights times |det J| for h = 1 (sum 1/2)
    double Me[2][6][6];         // int phi_a phi_b                  (scales h^2)
    double Ke[2][6][6];         // int grad phi_a . grad phi_b      (h-independent)
    double Se[2][12][12];       // int 2 D(phi_b e_d) : D(phi_a e_c), index c*6+a, d*6+b
    double Be[2][3][12];        // int psi_v d_d phi_b, index d*6+b (scales h)
    double Ge[3][3];            // Gamma edge: int phi_a phi_b      (scales h)
    double Gxe[3][3];           // Gamma edge: int phi_a d_x phi_b  (h-independent)
};

// Model coefficients of one run (Section 3.1 / Algorithm 3 notation).
struct Coef {
    double tau[3];              // phi_i C_i / dt
    double kap[3];              // k_i / mu_tilde
    double sst, s;              // sigma* k_f / mu_tilde, sigma k_m / mu_tilde
    double eta, nu, rho, dt;
    double beta;                // alpha nu / sqrt(k_F)
    double ctau;                // eta nu alpha sqrt(k_F) / mu_tilde
    int convection;
    int pad;
};

// One linear system family on a box of one grid (a local subdomain or the
// whole region of the coarse grid).
struct SysDesc {
    int kind;                   // KIND_POROUS (3 scalar fields) or KIND_OSEEN
    int region;
    int x0, y0, cx, cy;         // box origin / size in cells of its grid
    int N;                      // cells per axis of the region on that grid
    int gamma;                  // box touches Gamma
    int lw2, lh2, lw1, lh1;     // local lattice sizes
    int ndof, bw;               // unknowns and half-bandwidth of one band system
    int sub;                    // subdomain id, -1 for a coarse system
    int sample;                 // parameter sample of the system (coefficients, background fields)
    double h;
    long long band_off;         // band offset of field 0 (porous field f at + f*band_size)
    long long band_size;        // ndof * (2 bw + 1)
    long long dof_off;          // vector offset of field 0 (porous field f at + f*ndof)
    long long node_off;         // offset of the local P2 lattice in cls2/dof2
    long long vert_off;         // offset of the local P1 lattice in cls1/dof1
    long long e2_off;           // state offset (local P2 lattice); porous field f / velocity comp c at + f*lw2*lh2
    long long e1_off;           // state offset (local P1 lattice), conduit only
    long long zo;               // offset of the sample's block in the per-sample field arena (doubles)
};

// Host plan of a run: meshes, partition, per-system tables.
struct Plan {
    int NH, Nh, k;              // coarse / fine cells per unit length, refinement
    int nsx, nsy, overlap;
    std::vector<int> cuts[2][2];            // [region][axis]
    std::vector<SysDesc> por, ose;          // local systems
    SysDesc cpor, cns;                      // coarse systems (whole regions of T_H)
    std::vector<int8_t> cls2, cls1;         // per local lattice node: 0 free, 1 physical, 2 artificial
    std::vector<int32_t> dof2, dof1;        // unknown index or -1
    long long band_total_por = 0, band_total_ose = 0;
    long long dof_total_por = 0, dof_total_ose = 0;
    long long e2_total = 0, e1_total = 0;
    long long cband_por = 0, cband_ns = 0;
    // merge tables per region and axis: first owning core and owner count, P2 (2N+1) / P1 (N+1)
    std::vector<int32_t> own2_lo[2][2], own2_n[2][2], own1_lo[2][2], own1_n[2][2];
    int64_t local_dofs = 0;
    int max_bw = 0;
    // Strips of the local Oseen boxes for the Krylov path's preconditioner:
    // each conduit box cut along x into strips of at most strip_width cells
    // (cores of equal width, extended by strip_overlap cells into their
    // neighbours).  A strip is a box with the standard node classes, so its
    // faces inside the box are artificial (zero).  Per strip unknown, the
    // parent system's unknown (smap) and whether this strip owns it (sown:
    // its x lies in the strip's core; every parent unknown has one owner).
    std::vector<SysDesc> strip;
    std::vector<int32_t> strip_parent;      // index into ose
    std::vector<int32_t> smap;              // strip vector space -> parent unknown
    std::vector<int8_t> sown;
    long long band_total_strip = 0, dof_total_strip = 0;
    int strip_width = 0, strip_overlap = 0;
};

// plan.cpp
bool build_plan(const lp_mesh &m, const lp_partition &p, Plan &out, std::string &err);
// strips of every local Oseen box (appends their node tables); false if a
// strip's half-bandwidth exceeds max_bw
bool build_strips(Plan &P, int width, int overlap, int max_bw, std::string &err);

// fe.cpp: reference data and manufactured-solution data on a region lattice
void build_refdata(RefData &r);
// Spatial parts of the Example 1 exact fields on lattices of a grid with N
// cells: every exact field is a(x) cos t.  Output order: pF, pf, pm (porous
// P2 lattice), u1, u2 (conduit P2 lattice), p (conduit P1 lattice).
void exact_spatial(int N, std::vector<double> out[6]);
// Load vectors int q phi_a for the time-separable source terms of Example 1:
//   porous q_i = A_i cos t + B_i sin t      -> loads[i][0] (cos), loads[i][1] (sin), i = F,f,m
//   conduit f_c = -U_c sin t + (-nu lap U_c + d_c P) cos t + ((U.grad)U)_c cos^2 t
//                                           -> loads[3+c][0] (cos), [1] (sin), [2] (cos^2)
void source_loads(int N, const lp_params &prm, std::vector<double> loads[5][3]);

// The paper's own elements (Section 6): MINI in the conduit (P1 hats plus the
// bubble 27 l0 l1 l2, index 3), P1 porous pressures.  Unit-cell data as RefData.
constexpr int MINI_NQ = 25;  // collapsed Gauss 5 x 5, exact to degree 8
struct MiniRef {
    double w[MINI_NQ];               // weights times |det J| for h = 1 (sum 1/2)
    double phi[MINI_NQ][4];          // P1 hats (= the P1 pressure basis), then the bubble
    double dphi[2][MINI_NQ][4][2];   // unit-cell gradients per orientation
};
void build_mini_refdata(MiniRef &r);
// Loads of the Example 1 sources (time-separable parts as in source_loads)
// against P1 on the porous vertex lattice (loads[0..2][0..1], i + (N+1) j) and
// against MINI on the conduit (loads[3+c][0..2]: vertices, then one bubble per
// element id 2 (i + N j) + t).
void mini_source_loads(int N, const lp_params &prm, std::vector<double> loads[5][3]);
// Spatial parts of the Example 1 exact fields: pF, pf, pm, u1, u2, p at the
// vertices of their region, then u1, u2 at the element centroids.
void mini_exact_spatial(int N, std::vector<double> out[8]);
// Error status with a message for lp_last_error (api.cpp).
lp_status set_error(lp_status s, const std::string &msg);

}  // namespace lp
