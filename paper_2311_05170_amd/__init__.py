"""MI355X-native local parallel finite element stage (two-grid, overlapping
subdomains) for the transient triple-porosity Navier-Stokes model.

Importing the package loads nothing; ``paper_2311_05170_amd.lib`` binds the
C-ABI library ``liblp.so`` built by ``paper_2311_05170_amd.build``.
"""
