"""Uniform nested tetrahedral meshes and the 3D subdomain partition (Section 4
setting with d = 3: T_h a uniform refinement of T_H; Algorithm 3 Step 2).

Conventions (3D):
  * Each region is a unit cube split into N x N x N cells of size h = 1/N.
    The porous region Omega_p = (0,1)^3 sits below the conduit
    Omega_c = (0,1)^2 x (1,2); the interface Gamma is z = 1.
  * Cell (i, j, k) holds the six Kuhn tetrahedra about its (0,0,0)-(1,1,1)
    diagonal: for each permutation pi of (0, 1, 2), in lexicographic order,
    v0 = (i,j,k) and v_{m+1} = v_m + e_{pi(m)}.  Element id = 6 cell + rank(pi),
    cell = i + N (j + N k).  The split nests under integer refinement and
    cuts every face z = const along the (i,j)-(i+1,j+1) diagonal.
  * P2 nodes are the half-step lattice (a, b, c), 0 <= a, b, c <= 2N, index
    a + (2N+1)(b + (2N+1) c); in the conduit the vertical index counts up from
    Gamma.  P1 nodes are the vertices, index i + (N+1)(j + (N+1) k).
"""
import itertools

import numpy as np

from .fe3 import EDGES

POROUS, CONDUIT = 0, 1
PERMS = tuple(itertools.permutations(range(3)))       # lexicographic order


class RegionMesh3:
    """One region (porous or conduit) meshed with N^3 cells of six tetrahedra."""

    def __init__(self, N, region):
        self.N = int(N)
        self.h = 1.0 / self.N
        self.region = region
        self.z0 = 0.0 if region == POROUS else 1.0
        self.n2 = 2 * self.N + 1
        self.n1 = self.N + 1
        N = self.N
        I, J, K = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
        # cell order: i fastest, then j, then k
        I = I.transpose(2, 1, 0).ravel()
        J = J.transpose(2, 1, 0).ravel()
        K = K.transpose(2, 1, 0).ravel()
        nc = N ** 3
        ne = 6 * nc
        p2 = np.zeros((ne, 10), dtype=np.int64)
        p1 = np.zeros((ne, 4), dtype=np.int64)
        orient = np.zeros(ne, dtype=np.int64)
        cell = np.zeros((ne, 3), dtype=np.int64)
        L, L1 = self.n2, self.n1
        base = np.stack([I, J, K], 1)
        for r, pi in enumerate(PERMS):
            verts = [base.copy()]
            for m in range(3):
                v = verts[-1].copy()
                v[:, pi[m]] += 1
                verts.append(v)
            ids = 6 * np.arange(nc) + r
            for q in range(4):
                p1[ids, q] = verts[q][:, 0] + L1 * (verts[q][:, 1] + L1 * verts[q][:, 2])
                a = 2 * verts[q]
                p2[ids, q] = a[:, 0] + L * (a[:, 1] + L * a[:, 2])
            for e, (qa, qb) in enumerate(EDGES):
                a = verts[qa] + verts[qb]
                p2[ids, 4 + e] = a[:, 0] + L * (a[:, 1] + L * a[:, 2])
            orient[ids] = r
            cell[ids] = base
        self.el_p2, self.el_p1, self.el_orient, self.el_cell = p2, p1, orient, cell

    # --- coordinates ---------------------------------------------------------
    def p2_coords(self):
        a = np.arange(self.n2)
        A, B, C = np.meshgrid(a, a, a, indexing="ij")
        A, B, C = (X.transpose(2, 1, 0).ravel() for X in (A, B, C))
        return np.stack([A * self.h / 2, B * self.h / 2, self.z0 + C * self.h / 2], 1)

    def p1_coords(self):
        i = np.arange(self.n1)
        A, B, C = np.meshgrid(i, i, i, indexing="ij")
        A, B, C = (X.transpose(2, 1, 0).ravel() for X in (A, B, C))
        return np.stack([A * self.h, B * self.h, self.z0 + C * self.h], 1)

    def jacobian(self, r):
        """Affine map x = v0 + J xi of orientation r (columns: v1-v0, v2-v0, v3-v0)."""
        pi = PERMS[r]
        J = np.zeros((3, 3))
        v = np.zeros(3)
        for m in range(3):
            v[pi[m]] += 1
            J[:, m] = v
        return self.h * J

    def elements_in_box(self, x0, x1, y0, y1, z0, z1):
        """Ids of elements whose cell lies in [x0,x1) x [y0,y1) x [z0,z1)."""
        c = self.el_cell
        return np.nonzero((c[:, 0] >= x0) & (c[:, 0] < x1) & (c[:, 1] >= y0) & (c[:, 1] < y1) &
                          (c[:, 2] >= z0) & (c[:, 2] < z1))[0]

    def gamma_faces(self, x0=0, x1=None, y0=0, y1=None):
        """Interface triangles on Gamma for cells x0 <= i < x1, y0 <= j < y1:
        (n, 6) P2 node ids in the 2D P2 order (vertices, then midpoints of the
        edges (0,1), (1,2), (0,2)), the triangle orientation (0: {(i,j),
        (i+1,j), (i+1,j+1)}, 1: {(i,j), (i+1,j+1), (i,j+1)}) and the lower-left
        (x, y) corner."""
        N = self.N
        x1 = N if x1 is None else x1
        y1 = N if y1 is None else y1
        c = 2 * N if self.region == POROUS else 0
        L = self.n2

        def q(a, b):
            return a + L * (b + L * c)
        rows, ors, corners = [], [], []
        for j in range(y0, y1):
            for i in range(x0, x1):
                a, b = 2 * i, 2 * j
                rows.append([q(a, b), q(a + 2, b), q(a + 2, b + 2), q(a + 1, b), q(a + 2, b + 1), q(a + 1, b + 1)])
                ors.append(0)
                corners.append((i * self.h, j * self.h))
                rows.append([q(a, b), q(a + 2, b + 2), q(a, b + 2), q(a + 1, b + 1), q(a + 1, b + 2), q(a, b + 1)])
                ors.append(1)
                corners.append((i * self.h, j * self.h))
        return np.array(rows, dtype=np.int64), np.array(ors), np.array(corners)


class Subdomain3:
    """Omega_j (box in fine cells, region-relative) with its disjoint core D_j."""

    def __init__(self, sid, region, box, core, N):
        self.sid, self.region, self.N = sid, region, N
        self.x0, self.x1, self.y0, self.y1, self.z0, self.z1 = box
        self.d = core

    @property
    def touches_gamma(self):
        return self.z1 == self.N if self.region == POROUS else self.z0 == 0

    def p2_nodes(self, mesh):
        """Region P2 ids of the local lattice, local lexicographic order (x fastest)."""
        a = np.arange(2 * self.x0, 2 * self.x1 + 1)
        b = np.arange(2 * self.y0, 2 * self.y1 + 1)
        c = np.arange(2 * self.z0, 2 * self.z1 + 1)
        C, B, A = np.meshgrid(c, b, a, indexing="ij")
        A, B, C = A.ravel(), B.ravel(), C.ravel()
        return A + mesh.n2 * (B + mesh.n2 * C), A, B, C

    def p1_nodes(self, mesh):
        i = np.arange(self.x0, self.x1 + 1)
        j = np.arange(self.y0, self.y1 + 1)
        k = np.arange(self.z0, self.z1 + 1)
        C, B, A = np.meshgrid(k, j, i, indexing="ij")
        A, B, C = A.ravel(), B.ravel(), C.ravel()
        return A + mesh.n1 * (B + mesh.n1 * C), A, B, C

    def artificial_p1(self, I, J, K):
        """Mask of P1 vertices (region coordinates I, J, K) on an artificial face."""
        art = np.zeros(I.shape, dtype=bool)
        for lo, hi, X in ((self.x0, self.x1, I), (self.y0, self.y1, J), (self.z0, self.z1, K)):
            if lo > 0:
                art |= X == lo
            if hi < self.N:
                art |= X == hi
        return art

    def classify_p2(self, mesh):
        """Per local P2 node: 0 free, 1 physical Dirichlet, 2 artificial.
        Physical boundary = region boundary minus Gamma; artificial = the
        faces of Omega_j inside the region; a node on both is physical."""
        _, A, B, C = self.p2_nodes(mesh)
        N2 = 2 * self.N
        phys = (A == 0) | (A == N2) | (B == 0) | (B == N2)
        phys |= (C == 0) if self.region == POROUS else (C == N2)
        art = np.zeros_like(phys)
        for lo, hi, X in ((self.x0, self.x1, A), (self.y0, self.y1, B), (self.z0, self.z1, C)):
            if lo > 0:
                art |= X == 2 * lo
            if hi < self.N:
                art |= X == 2 * hi
        cls = np.where(phys, 1, np.where(art, 2, 0))
        return cls.astype(np.int64)


def uniform_cuts(N, nsub):
    assert N % nsub == 0
    return [k * (N // nsub) for k in range(nsub + 1)]


def make_subdomains3(N, cuts, overlap):
    """Subdomains of both regions.  cuts: {(region, axis): [0, ..., N]} for
    axes 0, 1, 2 (x, y, vertical); overlap: cells added on each side of a core
    (an int, or a per-axis triple), clipped to the region.  Ids: porous first,
    x fastest, then y, then vertical; conduit after."""
    ov = (overlap,) * 3 if np.isscalar(overlap) else tuple(overlap)
    subs = []
    sid = 0
    for region in (POROUS, CONDUIT):
        cx, cy, cz = cuts[(region, 0)], cuts[(region, 1)], cuts[(region, 2)]
        for kz in range(len(cz) - 1):
            for ky in range(len(cy) - 1):
                for kx in range(len(cx) - 1):
                    core = (cx[kx], cx[kx + 1], cy[ky], cy[ky + 1], cz[kz], cz[kz + 1])
                    box = (max(0, core[0] - ov[0]), min(N, core[1] + ov[0]),
                           max(0, core[2] - ov[1]), min(N, core[3] + ov[1]),
                           max(0, core[4] - ov[2]), min(N, core[5] + ov[2]))
                    subs.append(Subdomain3(sid, region, box, core, N))
                    sid += 1
    return subs


def extend_core(core, region_box):
    """Algorithm 3 Step 2 as the paper's examples apply it: a core box D,
    (x0, x1, y0, y1, z0, z1) in any units, extended on every side by half its
    own extent along that axis and clipped to its region's box."""
    out = []
    for ax in range(3):
        lo, hi = core[2 * ax], core[2 * ax + 1]
        half = (hi - lo) / 2
        out += [max(region_box[2 * ax], lo - half), min(region_box[2 * ax + 1], hi + half)]
    return tuple(out)
