"""Plain FP64 CPU oracle for the two-grid local parallel finite element method
(transient triple-porosity Navier-Stokes, Algorithm 3 of the paper, Section 5).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call, link
or execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (no kernels, headers, tables or pre/post-processing); both sides
receive the same plain inputs (mesh sizes, partition, parameters) from the
seeded workload generator.

Layout
  fe       quadrature rules and P1/P2 Lagrange bases on the reference triangle
  mesh     uniform right-triangle meshes, P2/P1 lattices, subdomain partitions
  mms      manufactured solution of Example 1 (Section 6) and derived data
  forms    the bilinear/trilinear forms of Section 3.1 assembled with scipy.sparse
  scheme   Algorithm 3: coarse decoupled step (Step 1), local corrections
           (Step 3), partition-of-unity correction (Step 4); Algorithm 1 on T_h
  fe3, mesh3, forms3, mms3, scheme3
           the same in 3D (Kuhn tetrahedra, Example 2 reflected): Algorithms 1
           and 3, exact prolongation, the Step 2 extension rule
  mini     the paper's own elements (MINI conduit, P1 porous; Section 6) with
           Algorithm 1 on one grid and Algorithm 3 (Steps 1-4)

Readings of points where the paper is silent are listed in the docstrings of
``scheme.py`` and, for the MINI element, ``mini.py``; every oracle function
cites the passage it follows.
"""
