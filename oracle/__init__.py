"""CPU oracle for the charge-conservation Nernst-Planck DG scheme (TEST INFRASTRUCTURE).

This package is test infrastructure only.  It may be imported by `tests/`, by
`__graft_entry__.smoke()` and by the `cpu_baseline` leg of `bench.py`, never by
the product path (`paper_2112_09271_amd`).  It shares no code with the GPU
library: every table, index map and formula here is written independently, in
plain float64 NumPy/SciPy (SymPy for manufactured sources), with element- and
face-vectorised full tabulations (no sum factorisation).

Contents (paper passages followed):
  quadrature  Gauss-Legendre and Gauss-Lobatto points, Lagrange tabulations
              (tensor-product elements with over-integration, Sec. 4 intro)
  mesh        structured box mesh, DOF indexing, face lists
  problem     species constants of the CNP model (Eq. charge2, nondim. Sec. 2.3),
              velocity fields, boundary data, manufactured sources
  dg          residual of the DG scheme (Eqs. NPDG / chargeDG), its exact
              Jacobian (apply + sparse assembly), d/d(boundary data), d/dPe,
              outflow-flux objective
  solve       initial guess (Sec. 4.3), Newton with backtracking and direct
              sparse solves (Sec. 4), adjoint by transposed LU, L2 errors

Pins (tests/test_oracle_*.py): quadrature closed forms and exactness,
polynomial consistency (exact solution in V_h gives a zero residual),
manufactured-solution L2 rates, SIPG symmetry of the potential block,
electroneutrality of the recovered c_m, global species balance, Jacobian vs
central differences of the residual, adjoint gradients vs central differences.
"""
