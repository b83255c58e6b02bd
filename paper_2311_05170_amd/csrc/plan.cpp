// Host planner: nested lattice meshes, the overlapping partition of
// Algorithm 3 Step 2, node classes (free / physical Dirichlet / artificial),
// the band ordering of every local system and the merge tables.
#include <algorithm>
#include <cstdlib>
#include <sstream>

#include "lp_internal.h"

namespace lp {

namespace {

// Class of a local P2 node at region half-lattice (A, B) for a box of a
// region with N cells: 1 physical boundary (region boundary minus Gamma),
// 2 artificial face (a face of the box strictly inside the region), 0 free.
// A node on both takes the physical class.
int8_t class_p2(int region, int N, int x0, int x1, int y0, int y1, int A, int B) {
    const int N2 = 2 * N;
    bool phys = (A == 0) || (A == N2) || (region == POROUS ? (B == 0) : (B == N2));
    if (phys) return 1;
    bool art = (x0 > 0 && A == 2 * x0) || (x1 < N && A == 2 * x1) ||
               (y0 > 0 && B == 2 * y0) || (y1 < N && B == 2 * y1);
    return art ? 2 : 0;
}

// P1 vertex class: 2 on an artificial face, else 0 (the pressure has no
// physical boundary condition).
int8_t class_p1(int N, int x0, int x1, int y0, int y1, int I, int J) {
    bool art = (x0 > 0 && I == x0) || (x1 < N && I == x1) || (y0 > 0 && J == y0) || (y1 < N && J == y1);
    return art ? 2 : 0;
}

// Fill node tables and band numbering of one system; returns ndof, sets bw.
void number_system(SysDesc &s, std::vector<int8_t> &cls2, std::vector<int32_t> &dof2,
                   std::vector<int8_t> &cls1, std::vector<int32_t> &dof1) {
    const int x1 = s.x0 + s.cx, y1 = s.y0 + s.cy;
    s.lw2 = 2 * s.cx + 1;
    s.lh2 = 2 * s.cy + 1;
    s.lw1 = s.cx + 1;
    s.lh1 = s.cy + 1;
    s.node_off = (long long)cls2.size();
    s.vert_off = (long long)cls1.size();
    const int n2 = s.lw2 * s.lh2, n1 = s.lw1 * s.lh1;
    cls2.resize(cls2.size() + n2);
    dof2.resize(dof2.size() + n2, -1);
    cls1.resize(cls1.size() + n1);
    dof1.resize(dof1.size() + n1, -1);
    int8_t *c2 = cls2.data() + s.node_off;
    int32_t *d2 = dof2.data() + s.node_off;
    int8_t *c1 = cls1.data() + s.vert_off;
    int32_t *d1 = dof1.data() + s.vert_off;
    for (int b = 0; b < s.lh2; ++b)
        for (int a = 0; a < s.lw2; ++a)
            c2[a + s.lw2 * b] = class_p2(s.region, s.N, s.x0, x1, s.y0, y1, 2 * s.x0 + a, 2 * s.y0 + b);
    for (int j = 0; j < s.lh1; ++j)
        for (int i = 0; i < s.lw1; ++i)
            c1[i + s.lw1 * j] = class_p1(s.N, s.x0, x1, s.y0, y1, s.x0 + i, s.y0 + j);
    int nd = 0;
    if (s.kind == KIND_POROUS) {
        for (int q = 0; q < n2; ++q)
            if (c2[q] == 0) d2[q] = nd++;
    } else {
        // Interleaved band order by lattice rows: (u_x, u_y) of each free node,
        // then the pressure of a vertex at that node.  Vertices of the first
        // lattice row wait until the velocity of their upper-right midpoint,
        // so that every pressure pivot meets an eliminated velocity coupling.
        auto put_p = [&](int a, int b) {
            int q = a / 2 + s.lw1 * (b / 2);
            if (c1[q] == 0 && d1[q] < 0) d1[q] = nd++;
        };
        for (int b = 0; b < s.lh2; ++b)
            for (int a = 0; a < s.lw2; ++a) {
                int q = a + s.lw2 * b;
                if (c2[q] == 0) { d2[q] = nd; nd += 2; }
                if (b > 0 && (a % 2 == 0) && (b % 2 == 0)) put_p(a, b);
                if (b == 1) {
                    if (a % 2 == 1) put_p(a - 1, 0);
                    if (a == s.lw2 - 1) put_p(a, 0);
                }
            }
    }
    s.ndof = nd;
    // half-bandwidth: max |i - j| over unknowns coupled through an element
    int bw = 0;
    for (int cj = 0; cj < s.cy; ++cj)
        for (int ci = 0; ci < s.cx; ++ci)
            for (int t = 0; t < 2; ++t) {
                int lo = 1 << 30, hi = -1;
                for (int k = 0; k < 6; ++k) {
                    int q = (2 * ci + off2a(t, k)) + s.lw2 * (2 * cj + off2b(t, k));
                    if (d2[q] >= 0) {
                        lo = std::min(lo, d2[q]);
                        hi = std::max(hi, d2[q] + (s.kind == KIND_OSEEN ? 1 : 0));
                    }
                }
                if (s.kind == KIND_OSEEN)
                    for (int k = 0; k < 3; ++k) {
                        int q = (ci + off1a(t, k)) + s.lw1 * (cj + off1b(t, k));
                        if (d1[q] >= 0) { lo = std::min(lo, d1[q]); hi = std::max(hi, d1[q]); }
                    }
                if (hi >= 0) bw = std::max(bw, hi - lo);
            }
    s.bw = bw;
    s.band_size = (long long)nd * (2 * bw + 1);
}

bool check_cuts(const std::vector<int> &c, int N, int n) {
    if ((int)c.size() != n + 1 || c.front() != 0 || c.back() != N) return false;
    for (int i = 0; i < n; ++i)
        if (c[i + 1] <= c[i]) return false;
    return true;
}

}  // namespace

bool build_plan(const lp_mesh &m, const lp_partition &p, Plan &P, std::string &err) {
    std::ostringstream e;
    if (m.dim != 2) { err = "only dim = 2 is implemented"; return false; }
    if (m.n_coarse < 1 || m.refine < 1) { err = "n_coarse and refine must be >= 1"; return false; }
    if ((long long)m.n_coarse * m.refine > 4096) { err = "fine grid larger than 4096 cells per axis"; return false; }
    if (p.nsub[0] < 1 || p.nsub[1] < 1 || p.overlap < 0) { err = "nsub must be >= 1 and overlap >= 0"; return false; }
    P.NH = m.n_coarse;
    P.k = m.refine;
    P.Nh = m.n_coarse * m.refine;
    P.nsx = p.nsub[0];
    P.nsy = p.nsub[1];
    P.overlap = p.overlap;
    const int N = P.Nh;
    int pos = 0;
    for (int r = 0; r < 2; ++r)
        for (int ax = 0; ax < 2; ++ax) {
            int n = ax == 0 ? P.nsx : P.nsy;
            std::vector<int> c(n + 1);
            if (p.cuts) {
                for (int i = 0; i <= n; ++i) c[i] = p.cuts[pos + i];
                pos += n + 1;
            } else {
                if (N % n != 0) { err = "uniform cuts need nsub to divide the fine cell count"; return false; }
                for (int i = 0; i <= n; ++i) c[i] = i * (N / n);
            }
            if (!check_cuts(c, N, n)) { err = "cuts must increase from 0 to N"; return false; }
            P.cuts[r][ax] = c;
        }
    P.cls2.clear(); P.dof2.clear(); P.cls1.clear(); P.dof1.clear();
    P.por.clear(); P.ose.clear();
    long long band_p = 0, band_o = 0, dof_p = 0, dof_o = 0, e2 = 0, e1 = 0;
    int sid = 0;
    P.local_dofs = 0;
    P.max_bw = 0;
    for (int r = 0; r < 2; ++r) {
        const auto &cx = P.cuts[r][0], &cy = P.cuts[r][1];
        for (int ky = 0; ky < P.nsy; ++ky)
            for (int kx = 0; kx < P.nsx; ++kx, ++sid) {
                SysDesc s{};
                s.kind = r == POROUS ? KIND_POROUS : KIND_OSEEN;
                s.region = r;
                int x0 = std::max(0, cx[kx] - P.overlap), x1 = std::min(N, cx[kx + 1] + P.overlap);
                int y0 = std::max(0, cy[ky] - P.overlap), y1 = std::min(N, cy[ky + 1] + P.overlap);
                s.x0 = x0; s.y0 = y0; s.cx = x1 - x0; s.cy = y1 - y0;
                s.N = N;
                s.h = 1.0 / N;
                s.gamma = r == POROUS ? (y1 == N) : (y0 == 0);
                s.sub = sid;
                number_system(s, P.cls2, P.dof2, P.cls1, P.dof1);
                if (s.kind == KIND_POROUS) {
                    s.band_off = band_p; band_p += 3 * s.band_size;
                    s.dof_off = dof_p; dof_p += 3LL * s.ndof;
                    s.e2_off = e2; e2 += 3LL * s.lw2 * s.lh2;
                    s.e1_off = 0;
                    P.local_dofs += 3LL * s.ndof;
                    P.por.push_back(s);
                } else {
                    s.band_off = band_o; band_o += s.band_size;
                    s.dof_off = dof_o; dof_o += s.ndof;
                    s.e2_off = e2; e2 += 2LL * s.lw2 * s.lh2;
                    s.e1_off = e1; e1 += (long long)s.lw1 * s.lh1;
                    P.local_dofs += s.ndof;
                    P.ose.push_back(s);
                }
                P.max_bw = std::max(P.max_bw, s.bw);
            }
    }
    P.band_total_por = band_p; P.band_total_ose = band_o;
    P.dof_total_por = dof_p; P.dof_total_ose = dof_o;
    P.e2_total = e2; P.e1_total = e1;
    // coarse systems: the whole regions of T_H
    for (int r = 0; r < 2; ++r) {
        SysDesc s{};
        s.kind = r == POROUS ? KIND_POROUS : KIND_OSEEN;
        s.region = r;
        s.x0 = 0; s.y0 = 0; s.cx = P.NH; s.cy = P.NH;
        s.N = P.NH;
        s.h = 1.0 / P.NH;
        s.gamma = 1;
        s.sub = -1;
        number_system(s, P.cls2, P.dof2, P.cls1, P.dof1);
        s.band_off = 0;
        s.dof_off = 0;
        s.e2_off = 0;
        s.e1_off = 0;
        if (r == POROUS) { P.cpor = s; P.cband_por = 3 * s.band_size; }
        else { P.cns = s; P.cband_ns = s.band_size; }
    }
    // merge tables: owners of each lattice coordinate among the closed cores
    for (int r = 0; r < 2; ++r)
        for (int ax = 0; ax < 2; ++ax) {
            const auto &c = P.cuts[r][ax];
            int n = (int)c.size() - 1;
            auto fill = [&](int npts, int scale, std::vector<int32_t> &lo, std::vector<int32_t> &cnt) {
                lo.assign(npts, -1);
                cnt.assign(npts, 0);
                for (int a = 0; a < npts; ++a)
                    for (int kk = 0; kk < n; ++kk)
                        if (a >= scale * c[kk] && a <= scale * c[kk + 1]) {
                            if (lo[a] < 0) lo[a] = kk;
                            cnt[a]++;
                        }
            };
            fill(2 * N + 1, 2, P.own2_lo[r][ax], P.own2_n[r][ax]);
            fill(N + 1, 1, P.own1_lo[r][ax], P.own1_n[r][ax]);
        }
    return true;
}

bool build_strips(Plan &P, int width, int overlap, int max_bw, std::string &err) {
    if (width < 2 * overlap + 1 || overlap < 1) { err = "strip width must exceed twice the strip overlap (>= 1)"; return false; }
    P.strip.clear(); P.strip_parent.clear(); P.smap.clear(); P.sown.clear();
    P.strip_width = width;
    P.strip_overlap = overlap;
    long long band = 0, dof = 0;
    for (int j = 0; j < (int)P.ose.size(); ++j) {
        const SysDesc &par = P.ose[j];
        const int w = par.cx;
        const int ns = w <= width ? 1 : (w + (width - 2 * overlap) - 1) / (width - 2 * overlap);
        for (int k = 0; k < ns; ++k) {
            // core [c0, c1) in box cells, equal widths (remainder to the first cores)
            const int c0 = par.x0 + (int)((long long)w * k / ns), c1 = par.x0 + (int)((long long)w * (k + 1) / ns);
            const int s0 = std::max(par.x0, c0 - (ns > 1 ? overlap : 0));
            const int s1 = std::min(par.x0 + par.cx, c1 + (ns > 1 ? overlap : 0));
            SysDesc s = par;
            s.x0 = s0;
            s.cx = s1 - s0;
            s.sub = j;
            number_system(s, P.cls2, P.dof2, P.cls1, P.dof1);
            if (s.bw > max_bw) {
                std::ostringstream e;
                e << "strip half-bandwidth " << s.bw << " exceeds " << max_bw;
                err = e.str();
                return false;
            }
            s.band_off = band; band += s.band_size;
            s.dof_off = dof; dof += s.ndof;
            s.e2_off = 0; s.e1_off = 0;
            // unknown maps: strip node (a, b) sits at parent lattice (a + 2 (s0 - x0), b)
            P.smap.resize(dof, -1);
            P.sown.resize(dof, 0);
            const int da = 2 * (s0 - par.x0);
            const bool last = k == ns - 1;
            auto owned = [&](int A) { return A >= 2 * c0 && (last ? A <= 2 * c1 : A < 2 * c1); };
            for (int b = 0; b < s.lh2; ++b)
                for (int a = 0; a < s.lw2; ++a) {
                    const int ds = P.dof2[s.node_off + a + s.lw2 * b];
                    if (ds < 0) continue;
                    const int dp = P.dof2[par.node_off + (a + da) + par.lw2 * b];
                    if (dp < 0) { err = "strip unknown without a parent unknown"; return false; }
                    const bool own = owned(2 * s0 + a);
                    for (int c = 0; c < 2; ++c) {
                        P.smap[s.dof_off + ds + c] = dp + c;
                        P.sown[s.dof_off + ds + c] = own;
                    }
                }
            for (int jj = 0; jj < s.lh1; ++jj)
                for (int i = 0; i < s.lw1; ++i) {
                    const int ds = P.dof1[s.vert_off + i + s.lw1 * jj];
                    if (ds < 0) continue;
                    const int dp = P.dof1[par.vert_off + (i + da / 2) + par.lw1 * jj];
                    if (dp < 0) { err = "strip unknown without a parent unknown"; return false; }
                    P.smap[s.dof_off + ds] = dp;
                    P.sown[s.dof_off + ds] = owned(2 * (s0 + i));
                }
            P.strip.push_back(s);
            P.strip_parent.push_back(j);
        }
    }
    P.band_total_strip = band;
    P.dof_total_strip = dof;
    // every parent unknown has exactly one owning strip
    std::vector<int> owners(P.dof_total_ose, 0);
    for (size_t si = 0; si < P.strip.size(); ++si) {
        const SysDesc &s = P.strip[si];
        const long long base = P.ose[P.strip_parent[si]].dof_off;
        for (int d = 0; d < s.ndof; ++d)
            if (P.sown[s.dof_off + d]) owners[base + P.smap[s.dof_off + d]]++;
    }
    for (long long i = 0; i < P.dof_total_ose; ++i)
        if (owners[i] != 1) { err = "strip ownership is not a partition of the local unknowns"; return false; }
    return true;
}

}  // namespace lp
