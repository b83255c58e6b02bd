"""Uniform nested meshes and the subdomain partition (Section 4 setting: T_h is a
uniform refinement of T_H; Algorithm 3 Step 2: disjoint D_j enlarged to
overlapping Omega_j aligned with T_h).

Conventions (2D):
  * Each region is a unit square split into N x N cells of size h = 1/N.  The
    porous region Omega_p = (0,1)^2 sits below the conduit Omega_c = (0,1)x(1,2);
    the interface Gamma is y = 1 (Example 1 of Section 6).
  * Cell (i, j) holds two right triangles:
      T0 = {(i,j), (i+1,j), (i+1,j+1)},  T1 = {(i,j), (i+1,j+1), (i,j+1)};
    element id = 2 (i + N j) + t.  Both nest under integer refinement.
  * P2 nodes are the half-step lattice (a, b), 0 <= a, b <= 2N, index
    a + (2N+1) b; in the conduit the vertical index counts up from Gamma.
    P1 nodes are the vertices (i, j), index i + (N+1) j.
"""
import numpy as np

POROUS, CONDUIT = 0, 1


class RegionMesh:
    """One region (porous or conduit) meshed with N x N cells."""

    def __init__(self, N, region):
        self.N = int(N)
        self.h = 1.0 / self.N
        self.region = region
        self.y0 = 0.0 if region == POROUS else 1.0
        self.n2 = 2 * self.N + 1          # P2 lattice points per axis
        self.n1 = self.N + 1              # P1 lattice points per axis
        N = self.N
        ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
        ii = ii.ravel(); jj = jj.ravel()   # cell order: i fastest
        ne = 2 * N * N
        p2 = np.zeros((ne, 6), dtype=np.int64)
        p1 = np.zeros((ne, 3), dtype=np.int64)
        orient = np.zeros(ne, dtype=np.int64)
        cell = np.zeros((ne, 2), dtype=np.int64)
        L = self.n2

        def q(a, b):
            return a + L * b

        def v(i, j):
            return i + self.n1 * j

        a, b = 2 * ii, 2 * jj
        e0 = 2 * (ii + N * jj)
        e1 = e0 + 1
        # T0: (0,0) (1,0) (1,1); midpoints (0,1),(1,2),(0,2) of the local vertices
        p2[e0] = np.stack([q(a, b), q(a + 2, b), q(a + 2, b + 2),
                           q(a + 1, b), q(a + 2, b + 1), q(a + 1, b + 1)], 1)
        p1[e0] = np.stack([v(ii, jj), v(ii + 1, jj), v(ii + 1, jj + 1)], 1)
        # T1: (0,0) (1,1) (0,1)
        p2[e1] = np.stack([q(a, b), q(a + 2, b + 2), q(a, b + 2),
                           q(a + 1, b + 1), q(a + 1, b + 2), q(a, b + 1)], 1)
        p1[e1] = np.stack([v(ii, jj), v(ii + 1, jj + 1), v(ii, jj + 1)], 1)
        orient[e1] = 1
        cell[e0] = np.stack([ii, jj], 1)
        cell[e1] = np.stack([ii, jj], 1)
        self.el_p2, self.el_p1, self.el_orient, self.el_cell = p2, p1, orient, cell

    # --- coordinates ---------------------------------------------------------
    def p2_coords(self):
        a, b = np.meshgrid(np.arange(self.n2), np.arange(self.n2), indexing="xy")
        return np.stack([a.ravel() * self.h / 2, self.y0 + b.ravel() * self.h / 2], 1)

    def p1_coords(self):
        i, j = np.meshgrid(np.arange(self.n1), np.arange(self.n1), indexing="xy")
        return np.stack([i.ravel() * self.h, self.y0 + j.ravel() * self.h], 1)

    def jacobian(self, t):
        """Affine map x = v0 + J xi of orientation t (both have det J = h^2)."""
        h = self.h
        if t == 0:
            return h * np.array([[1.0, 1.0], [0.0, 1.0]])
        return h * np.array([[1.0, 0.0], [1.0, 1.0]])

    def elements_in_box(self, x0, x1, y0, y1):
        """Ids of elements whose cell lies in [x0,x1) x [y0,y1)."""
        ci, cj = self.el_cell[:, 0], self.el_cell[:, 1]
        return np.nonzero((ci >= x0) & (ci < x1) & (cj >= y0) & (cj < y1))[0]

    def gamma_edges(self, x0=0, x1=None):
        """Interface edges on Gamma for cells x0 <= i < x1: (n, 3) P2 node ids
        (end at x_i, midpoint, end at x_{i+1}) and the left x coordinate."""
        if x1 is None:
            x1 = self.N
        i = np.arange(x0, x1)
        b = 2 * self.N if self.region == POROUS else 0
        nodes = np.stack([2 * i + self.n2 * b, 2 * i + 1 + self.n2 * b,
                          2 * i + 2 + self.n2 * b], 1)
        return nodes, i * self.h


class Subdomain:
    """Omega_j (box in fine cells, region-relative) with its disjoint core D_j."""

    def __init__(self, sid, region, box, core, N):
        self.sid, self.region, self.N = sid, region, N
        self.x0, self.x1, self.y0, self.y1 = box
        self.d = core
        self.touches_gamma = (self.y1 == N) if region == POROUS else (self.y0 == 0)

    def p2_nodes(self, mesh):
        """Region P2 ids of the local lattice, local lexicographic order (x fastest)."""
        a = np.arange(2 * self.x0, 2 * self.x1 + 1)
        b = np.arange(2 * self.y0, 2 * self.y1 + 1)
        A, B = np.meshgrid(a, b, indexing="xy")
        return (A + mesh.n2 * B).ravel(), A.ravel(), B.ravel()

    def p1_nodes(self, mesh):
        i = np.arange(self.x0, self.x1 + 1)
        j = np.arange(self.y0, self.y1 + 1)
        I, J = np.meshgrid(i, j, indexing="xy")
        return (I + mesh.n1 * J).ravel(), I.ravel(), J.ravel()

    def classify_p2(self, mesh):
        """Per local P2 node: 0 free, 1 physical Dirichlet, 2 artificial Dirichlet.

        Physical boundary = region boundary minus Gamma (Dirichlet, Section 2);
        artificial boundary = the faces of Omega_j inside the region
        (homogeneous Dirichlet for the local correction).  A node on both takes
        the physical value."""
        _, A, B = self.p2_nodes(mesh)
        N2 = 2 * self.N
        phys = (A == 0) | (A == N2)
        if self.region == POROUS:
            phys |= (B == 0)
        else:
            phys |= (B == N2)
        art = np.zeros_like(phys)
        if self.x0 > 0:
            art |= (A == 2 * self.x0)
        if self.x1 < self.N:
            art |= (A == 2 * self.x1)
        if self.y0 > 0:
            art |= (B == 2 * self.y0)
        if self.y1 < self.N:
            art |= (B == 2 * self.y1)
        cls = np.zeros(A.shape, dtype=np.int64)
        cls[art] = 2
        cls[phys] = 1
        return cls


    def artificial_p1(self, I, J):
        """Mask of P1 vertices (region coordinates I, J) on an artificial face."""
        art = np.zeros(I.shape, dtype=bool)
        if self.x0 > 0:
            art |= (I == self.x0)
        if self.x1 < self.N:
            art |= (I == self.x1)
        if self.y0 > 0:
            art |= (J == self.y0)
        if self.y1 < self.N:
            art |= (J == self.y1)
        return art


def uniform_cuts(N, nsub):
    """Uniform cut lattice c_k = k N / nsub (must be integral)."""
    assert N % nsub == 0
    return [k * N // nsub for k in range(nsub + 1)]


def make_subdomains(N, cuts, overlap):
    """Algorithm 3 Step 2 on one grid.

    cuts: dict {(region, axis): [c_0=0, ..., c_n=N]} in fine cells.  D_j is the
    tensor product of consecutive cuts; Omega_j = D_j enlarged by `overlap`
    fine cells per side, clipped to its region (never crossing Gamma).
    Ids: porous first, x fastest then y; conduit ids follow."""
    subs = []
    sid = 0
    for region in (POROUS, CONDUIT):
        cx, cy = cuts[(region, 0)], cuts[(region, 1)]
        for ky in range(len(cy) - 1):
            for kx in range(len(cx) - 1):
                core = (cx[kx], cx[kx + 1], cy[ky], cy[ky + 1])
                box = (max(0, cx[kx] - overlap), min(N, cx[kx + 1] + overlap),
                       max(0, cy[ky] - overlap), min(N, cy[ky + 1] + overlap))
                subs.append(Subdomain(sid, region, box, core, N))
                sid += 1
    return subs


def owner_counts(cuts_axis, coords_half):
    """Number of closed cores [c_k, c_{k+1}] containing each half-lattice coordinate."""
    c = np.asarray(cuts_axis) * 2
    cnt = np.zeros(len(coords_half), dtype=np.int64)
    for k in range(len(c) - 1):
        cnt += ((coords_half >= c[k]) & (coords_half <= c[k + 1])).astype(np.int64)
    return cnt
