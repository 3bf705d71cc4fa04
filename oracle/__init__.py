"""CPU FP64 oracle for the MDP domain-decomposition hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything from this package: only the tests, the package's smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the GPU library (no
kernels, headers, helpers, tables or constant generators); the only common
module is the seeded workload description, which holds none of the method's
arithmetic.

The oracle computes the plain definitions of what the method computes
(North, Tsynkov & Turkel, "Non-iterative domain decomposition for the
Helmholtz equation using the method of difference potentials"):

  grid.py        grid sets N0, M0, M+, N+, N-, gamma and the side of each
                 gamma node (Sec. 3.2.2)
  scheme.py      the compact fourth-order operator L^(h) (eq. FD_scheme) and
                 the assembled discrete auxiliary problem (eq. discrete_AP);
                 G^(h) by banded LU with partial pivoting (LAPACK gbtrf/gbtrs)
                 and, for large grids, by the separable route (explicit sine
                 sums + one tridiagonal LAPACK solve per mode); a brute-force
                 dense solve for tiny grids
  extension.py   Chebyshev basis on each side and the equation-based
                 extension Ex^(H) (Sec. 3.2.3-3.2.4)
  projector.py   Q = [(P_gamma - I) Ex Psi_j], one AP solve per column
                 (eq. Q_construction); explicit P_gamma for small grids
  interface.py   boundary and interface conditions eliminated in coefficient
                 space (Sec. 3.3.3), least squares by the oracle's own complex
                 Householder QR (Sec. 3.5 step 2)
  solve.py       reconstruction u = P_{N+} xi_gamma (eq. potential_solution_homo)
                 and the end-to-end domain-decomposition solve

Readings of points the paper leaves silent or prints garbled are stated in the
module that uses them.  Parity status: every function here is pinned by a
`-m "not gpu"` test against closed forms, invariants, brute force or the
paper's printed numbers, except the Sommerfeld-type end rows of the discrete
auxiliary problem, whose exact coefficients are a reading of a garbled
equation: their fourth-order consistency is pinned, their digits are
"parity unpinned" beyond that.
"""
