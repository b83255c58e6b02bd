// Reference-element data and manufactured-solution data (host, FP64).
//
// P2/P1 Lagrange bases on the reference triangle (0,0),(1,0),(0,1) with
// barycentrics l0 = 1 - xi - eta, l1 = xi, l2 = eta; P2 node order: vertices,
// then midpoints of edges (0,1), (1,2), (0,2).  Quadrature: the collapsed
// (Duffy) tensor Gauss-Legendre rule, exact to degree 2m - 2 on triangles.
// Gauss-Legendre nodes are found by Newton's method on the three-term
// Legendre recurrence.
#include <cmath>

#include "lp_internal.h"

namespace lp {

namespace {

const double PI = 3.14159265358979323846;

void gauss_legendre_01(int m, std::vector<double> &x, std::vector<double> &w) {
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int i = 0; i < m; ++i) {
        double z = std::cos(PI * (i + 0.75) / (m + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 1; j < m; ++j) {
                double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_m(z), p0 = P_{m-1}(z)
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = (1.0 - z) / 2.0;                 // map [-1,1] -> [0,1], ascending in i
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) halved for [0,1]
    }
}

void triangle_rule(int m, std::vector<double> &xi, std::vector<double> &eta, std::vector<double> &wt) {
    std::vector<double> g, w;
    gauss_legendre_01(m, g, w);
    xi.clear(); eta.clear(); wt.clear();
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            xi.push_back(g[i]);
            eta.push_back(g[j] * (1.0 - g[i]));
            wt.push_back(w[i] * w[j] * (1.0 - g[i]));
        }
}

void p2_eval(double xi, double eta, double v[6], double g[6][2]) {
    double l[3] = {1.0 - xi - eta, xi, eta};
    const double dl[3][2] = {{-1, -1}, {1, 0}, {0, 1}};
    for (int i = 0; i < 3; ++i) {
        v[i] = l[i] * (2 * l[i] - 1);
        for (int d = 0; d < 2; ++d) g[i][d] = (4 * l[i] - 1) * dl[i][d];
    }
    const int e[3][2] = {{0, 1}, {1, 2}, {0, 2}};
    for (int k = 0; k < 3; ++k) {
        int i = e[k][0], j = e[k][1];
        v[3 + k] = 4 * l[i] * l[j];
        for (int d = 0; d < 2; ++d) g[3 + k][d] = 4 * (l[i] * dl[j][d] + l[j] * dl[i][d]);
    }
}

// reference gradient -> physical gradient on the unit cell: g_x = g_xi J^{-1}
//   T0: J = [[1,1],[0,1]],  T1: J = [[1,0],[1,1]]
void to_physical(int t, const double gr[2], double gx[2]) {
    if (t == 0) { gx[0] = gr[0]; gx[1] = -gr[0] + gr[1]; }
    else { gx[0] = gr[0] - gr[1]; gx[1] = gr[1]; }
}

// affine map of orientation t on a cell with origin (X0, Y0) and size h
void to_xy(int t, double X0, double Y0, double h, double xi, double eta, double &x, double &y) {
    if (t == 0) { x = X0 + h * (xi + eta); y = Y0 + h * eta; }
    else { x = X0 + h * xi; y = Y0 + h * (xi + eta); }
}

inline double gfun(double x) { return 2.0 - PI * std::sin(PI * x); }
inline double gfun2(double x) { return PI * PI * PI * std::sin(PI * x); }       // g''
inline double gfun1(double x) { return -PI * PI * std::cos(PI * x); }           // g'

// Example 1 porous y-profiles Y_i (p_i = g(x) Y_i(y) cos t) and Y_i''
void yprof(int i, double y, double &Y, double &Y2) {
    if (i == 0) { Y = 1.0 - y - std::cos(PI * y); Y2 = PI * PI * std::cos(PI * y); }
    else if (i == 1) { Y = std::cos(PI * (1.0 - y)); Y2 = -PI * PI * std::cos(PI * (1.0 - y)); }
    else {
        double ph = 0.5 * PI * (3 * y * y * y - 2 * y * y);
        double p1 = 0.5 * PI * (9 * y * y - 4 * y);
        double p2 = 0.5 * PI * (18 * y - 4);
        Y = std::sin(ph);
        Y2 = std::cos(ph) * p2 - std::sin(ph) * p1 * p1;
    }
}


// Time-separable parts of the Example 1 sources at a point of a region
// (region-relative y): val[f][k] for f = F, f, m (porous: k = cos t, sin t) or
// f = 3 + c (conduit u_c: k = cos t, sin t, cos^2 t); unused parts stay 0.
void source_point(int region, double x, double yl, const lp_params &prm, double val[5][3]) {
    const double mu = prm.mu_tilde;
    const double kap[3] = {prm.k[0] / mu, prm.k[1] / mu, prm.k[2] / mu};
    const double sst = prm.sigma_star * prm.k[1] / mu, s = prm.sigma * prm.k[2] / mu;
    const double nu = prm.nu;
    for (int f = 0; f < 5; ++f)
        for (int k = 0; k < 3; ++k) val[f][k] = 0.0;
    if (region == POROUS) {
        double y = yl, a[3], lap[3];
        for (int f = 0; f < 3; ++f) {
            double Y, Y2;
            yprof(f, y, Y, Y2);
            a[f] = gfun(x) * Y;
            lap[f] = gfun2(x) * Y + gfun(x) * Y2;
        }
        // cos t parts (diffusion + exchange), sin t parts (-phi C a)
        val[0][0] = -kap[0] * lap[0] + sst * (a[0] - a[1]);
        val[1][0] = -kap[1] * lap[1] + sst * (a[1] - a[0]) + s * (a[1] - a[2]);
        val[2][0] = -kap[2] * lap[2] + s * (a[2] - a[1]);
        for (int f = 0; f < 3; ++f) val[f][1] = -prm.phi[f] * prm.C[f] * a[f];
    } else {
        double y = 1.0 + yl, ym = y - 1.0;
        double U1 = x * x * ym * ym + y;
        double U2 = -2.0 / 3.0 * x * ym * ym * ym + gfun(x);
        double U1x = 2 * x * ym * ym, U1y = 2 * x * x * ym + 1.0;
        double U2x = -2.0 / 3.0 * ym * ym * ym + gfun1(x), U2y = -2 * x * ym * ym;
        double L1 = 2 * ym * ym + 2 * x * x;
        double L2 = -4 * x * ym + gfun2(x);
        double Px = gfun1(x) * std::sin(0.5 * PI * y);
        double Py = gfun(x) * 0.5 * PI * std::cos(0.5 * PI * y);
        val[3][0] = -nu * L1 + Px;
        val[4][0] = -nu * L2 + Py;
        val[3][1] = -U1;
        val[4][1] = -U2;
        val[3][2] = U1 * U1x + U2 * U1y;
        val[4][2] = U1 * U2x + U2 * U2y;
    }
}

}  // namespace

void build_refdata(RefData &r) {
    std::vector<double> xi, eta, wt;
    triangle_rule(4, xi, eta, wt);   // 16 points, exact to degree 6
    for (int q = 0; q < NQ; ++q) {
        double v[6], g[6][2];
        p2_eval(xi[q], eta[q], v, g);
        r.w[q] = wt[q];              // |det J| = 1 on the unit cell
        for (int a = 0; a < 6; ++a) {
            r.phi[q][a] = v[a];
            for (int t = 0; t < 2; ++t) to_physical(t, g[a], r.dphi[t][q][a]);
        }
        r.psi[q][0] = 1.0 - xi[q] - eta[q];
        r.psi[q][1] = xi[q];
        r.psi[q][2] = eta[q];
    }
    for (int t = 0; t < 2; ++t) {
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) {
                double m = 0, k = 0;
                for (int q = 0; q < NQ; ++q) {
                    m += r.w[q] * r.phi[q][a] * r.phi[q][b];
                    k += r.w[q] * (r.dphi[t][q][a][0] * r.dphi[t][q][b][0] + r.dphi[t][q][a][1] * r.dphi[t][q][b][1]);
                }
                r.Me[t][a][b] = m;
                r.Ke[t][a][b] = k;
            }
        // S[(a,c),(b,d)] = delta_cd grad phi_a . grad phi_b + d_d phi_a d_c phi_b
        for (int c = 0; c < 2; ++c)
            for (int a = 0; a < 6; ++a)
                for (int d = 0; d < 2; ++d)
                    for (int b = 0; b < 6; ++b) {
                        double s = c == d ? r.Ke[t][a][b] : 0.0;
                        for (int q = 0; q < NQ; ++q) s += r.w[q] * r.dphi[t][q][a][d] * r.dphi[t][q][b][c];
                        r.Se[t][c * 6 + a][d * 6 + b] = s;
                    }
        for (int v = 0; v < 3; ++v)
            for (int d = 0; d < 2; ++d)
                for (int b = 0; b < 6; ++b) {
                    double s = 0;
                    for (int q = 0; q < NQ; ++q) s += r.w[q] * r.psi[q][v] * r.dphi[t][q][b][d];
                    r.Be[t][v][d * 6 + b] = s;
                }
    }
    std::vector<double> s, ws;
    gauss_legendre_01(6, s, ws);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double g = 0, gx = 0;
            for (int q = 0; q < 6; ++q) {
                double z = s[q];
                double val[3] = {(1 - z) * (1 - 2 * z), 4 * z * (1 - z), z * (2 * z - 1)};
                double der[3] = {4 * z - 3, 4 - 8 * z, 4 * z - 1};
                g += ws[q] * val[a] * val[b];
                gx += ws[q] * val[a] * der[b];
            }
            r.Ge[a][b] = g;
            r.Gxe[a][b] = gx;
        }
}

void exact_spatial(int N, std::vector<double> out[6]) {
    const int n2 = 2 * N + 1, n1 = N + 1;
    const double h = 1.0 / N;
    for (int f = 0; f < 3; ++f) out[f].assign((size_t)n2 * n2, 0.0);
    out[3].assign((size_t)n2 * n2, 0.0);
    out[4].assign((size_t)n2 * n2, 0.0);
    out[5].assign((size_t)n1 * n1, 0.0);
    for (int b = 0; b < n2; ++b)
        for (int a = 0; a < n2; ++a) {
            const size_t q = a + (size_t)n2 * b;
            double x = a * h / 2, y = b * h / 2;
            for (int f = 0; f < 3; ++f) {
                double Y, Y2;
                yprof(f, y, Y, Y2);
                out[f][q] = gfun(x) * Y;
            }
            double yc = 1.0 + y;
            out[3][q] = x * x * (yc - 1) * (yc - 1) + yc;
            out[4][q] = -2.0 / 3.0 * x * (yc - 1) * (yc - 1) * (yc - 1) + gfun(x);
        }
    for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
            double x = i * h, y = 1.0 + j * h;
            out[5][i + (size_t)n1 * j] = gfun(x) * std::sin(0.5 * PI * y);
        }
}

void source_loads(int N, const lp_params &prm, std::vector<double> loads[5][3]) {
    const int n2 = 2 * N + 1;
    const double h = 1.0 / N;
    for (int f = 0; f < 5; ++f)
        for (int k = 0; k < 3; ++k) loads[f][k].assign((size_t)n2 * n2, 0.0);
    std::vector<double> xi, eta, wt;
    triangle_rule(6, xi, eta, wt);   // 36 points, exact to degree 10
    const int nq = (int)xi.size();
    std::vector<double> phi(nq * 6);
    for (int q = 0; q < nq; ++q) {
        double v[6], g[6][2];
        p2_eval(xi[q], eta[q], v, g);
        for (int a = 0; a < 6; ++a) phi[q * 6 + a] = v[a];
    }
    for (int region = 0; region < 2; ++region)
        for (int cj = 0; cj < N; ++cj)
            for (int ci = 0; ci < N; ++ci)
                for (int t = 0; t < 2; ++t) {
                    double acc[5][3][6] = {};
                    for (int q = 0; q < nq; ++q) {
                        double x, yl;
                        to_xy(t, ci * h, cj * h, h, xi[q], eta[q], x, yl);
                        const double w = wt[q] * h * h;
                        double val[5][3];
                        source_point(region, x, yl, prm, val);
                        for (int f = 0; f < 5; ++f)
                            for (int k = 0; k < 3; ++k)
                                if (val[f][k] != 0.0)
                                    for (int a2 = 0; a2 < 6; ++a2) acc[f][k][a2] += w * val[f][k] * phi[q * 6 + a2];
                    }
                    for (int a2 = 0; a2 < 6; ++a2) {
                        size_t node = (2 * ci + off2a(t, a2)) + (size_t)n2 * (2 * cj + off2b(t, a2));
                        int f0 = region == POROUS ? 0 : 3, f1 = region == POROUS ? 3 : 5;
                        for (int f = f0; f < f1; ++f)
                            for (int k = 0; k < 3; ++k) loads[f][k][node] += acc[f][k][a2];
                    }
                }
}

// ---------------------------------------------------------------------------
// The paper's own elements (Section 6): MINI (P1 plus the cubic bubble
// 27 l0 l1 l2) in the conduit, P1 for the porous pressures.

void build_mini_refdata(MiniRef &r) {
    std::vector<double> xi, eta, wt;
    triangle_rule(5, xi, eta, wt);   // 25 points, exact to degree 8
    const double dl[3][2] = {{-1, -1}, {1, 0}, {0, 1}};
    for (int q = 0; q < MINI_NQ; ++q) {
        const double l[3] = {1.0 - xi[q] - eta[q], xi[q], eta[q]};
        r.w[q] = wt[q];
        double g[4][2];
        for (int a = 0; a < 3; ++a) {
            r.phi[q][a] = l[a];
            g[a][0] = dl[a][0];
            g[a][1] = dl[a][1];
        }
        r.phi[q][3] = 27.0 * l[0] * l[1] * l[2];
        for (int d = 0; d < 2; ++d)
            g[3][d] = 27.0 * (l[1] * l[2] * dl[0][d] + l[0] * l[2] * dl[1][d] + l[0] * l[1] * dl[2][d]);
        for (int t = 0; t < 2; ++t)
            for (int a = 0; a < 4; ++a) to_physical(t, g[a], r.dphi[t][q][a]);
    }
}

void mini_source_loads(int N, const lp_params &prm, std::vector<double> loads[5][3]) {
    const int n1 = N + 1;
    const size_t nv = (size_t)n1 * n1, ne = 2 * (size_t)N * N;
    const double h = 1.0 / N;
    for (int f = 0; f < 5; ++f)
        for (int k = 0; k < 3; ++k) loads[f][k].assign(f < 3 ? nv : nv + ne, 0.0);
    std::vector<double> xi, eta, wt;
    triangle_rule(6, xi, eta, wt);   // 36 points, exact to degree 10
    const int nq = (int)xi.size();
    for (int region = 0; region < 2; ++region)
        for (int cj = 0; cj < N; ++cj)
            for (int ci = 0; ci < N; ++ci)
                for (int t = 0; t < 2; ++t) {
                    double acc[5][3][4] = {};
                    for (int q = 0; q < nq; ++q) {
                        const double l[3] = {1.0 - xi[q] - eta[q], xi[q], eta[q]};
                        const double phi[4] = {l[0], l[1], l[2], 27.0 * l[0] * l[1] * l[2]};
                        double x, yl;
                        to_xy(t, ci * h, cj * h, h, xi[q], eta[q], x, yl);
                        const double w = wt[q] * h * h;
                        double val[5][3];
                        source_point(region, x, yl, prm, val);
                        for (int f = 0; f < 5; ++f)
                            for (int k = 0; k < 3; ++k)
                                if (val[f][k] != 0.0)
                                    for (int a = 0; a < 4; ++a) acc[f][k][a] += w * val[f][k] * phi[a];
                    }
                    const int f0 = region == POROUS ? 0 : 3, f1 = region == POROUS ? 3 : 5;
                    const size_t e = 2 * ((size_t)ci + (size_t)N * cj) + t;
                    for (int f = f0; f < f1; ++f)
                        for (int k = 0; k < 3; ++k) {
                            for (int a = 0; a < 3; ++a)
                                loads[f][k][(ci + off1a(t, a)) + (size_t)n1 * (cj + off1b(t, a))] += acc[f][k][a];
                            if (region == CONDUIT) loads[f][k][nv + e] += acc[f][k][3];
                        }
                }
}

void mini_exact_spatial(int N, std::vector<double> out[8]) {
    const int n1 = N + 1;
    const double h = 1.0 / N;
    for (int f = 0; f < 6; ++f) out[f].assign((size_t)n1 * n1, 0.0);
    for (int f = 6; f < 8; ++f) out[f].assign(2 * (size_t)N * N, 0.0);
    auto u = [](double x, double y, double &u1, double &u2) {
        const double ym = y - 1.0;
        u1 = x * x * ym * ym + y;
        u2 = -2.0 / 3.0 * x * ym * ym * ym + gfun(x);
    };
    for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n1; ++i) {
            const size_t v = i + (size_t)n1 * j;
            const double x = i * h, y = j * h;
            for (int f = 0; f < 3; ++f) {
                double Y, Y2;
                yprof(f, y, Y, Y2);
                out[f][v] = gfun(x) * Y;
            }
            u(x, 1.0 + y, out[3][v], out[4][v]);
            out[5][v] = gfun(x) * std::sin(0.5 * PI * (1.0 + y));
        }
    for (int cj = 0; cj < N; ++cj)
        for (int ci = 0; ci < N; ++ci)
            for (int t = 0; t < 2; ++t) {
                double x, yl;
                to_xy(t, ci * h, cj * h, h, 1.0 / 3.0, 1.0 / 3.0, x, yl);
                u(x, 1.0 + yl, out[6][2 * (ci + (size_t)N * cj) + t], out[7][2 * (ci + (size_t)N * cj) + t]);
            }
}

}  // namespace lp
