"""FP64 CPU oracle for the FAS / weighted-Schwarz DG-SEM hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or executes anything in this package; only the
test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.

It is a plain, slow, obviously-correct restatement of what the paper defines,
written in numpy/scipy in double precision and sharing no code with the GPU
path.  Every module cites the passage it follows:

* ``gll``       Gauss-Lobatto-Legendre nodes, weights, differentiation and
                interpolation matrices (Sec. 2.2, Remark on basis functions).
* ``mesh``      isoparametric geometry: metric, surface measure, normals,
                h_perp and the SIPG penalty (Sec. 2.2, eq. helmholtz:dgm).
* ``operator``  matrix-free SIPG operator, right-hand side, dense assembly
                (eq. helmholtz:dgm, eq. helmholtz:system).
* ``sipg1d``    1D SIPG matrices on uniform meshes (used for the Kronecker pin
                and for the 1D subdomain matrices of Sec. 4.3.1).
* ``schwarz``   surrogate cuboid, 1D face-condition variants, generalized
                eigenproblem, fast-diagonalisation solve, weighting, WAS
                (Sec. 4.3.1, eq. schwarz:tpo, eq. schwarz:correction, Alg. 5).
* ``unstructured`` Schwarz subdomains on unstructured meshes: walks across
                oriented faces (Sec. 5.1), zero fill and merging at irregular
                edges and vertices (Sec. 4.3.1, design principles 4-6).
* ``transfer``  embedded interpolation I, restriction R = I^T, projection P
                (Sec. 3.2).
* ``solvers``   SCG (Alg. 6), FAS V-cycle (Alg. 2), CS V-cycle (Alg. 1).
* ``dense``     brute-force dense versions of the above on tiny meshes.

Parity status of each function is stated in its docstring; functions that no
test pins against an independent fact say "parity unpinned".
"""
