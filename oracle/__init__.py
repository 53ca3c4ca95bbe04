"""FP64 CPU oracle for LOBPCG on the 7-point Laplacian -- TEST INFRASTRUCTURE.

This package is the independent reference that the GPU library is checked
against.  It is plain and slow on purpose.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the GPU
library's product path never does, and the two share no code.

Contents
  closed_form  the Laplacian's eigenvalues and sine eigenvectors (Section 4.1)
  grid         the grid operators (C loops in grid_ops.c, via ctypes): the
               7-point and variable-coefficient operators, Jacobi sweep,
               full-weighting restriction, trilinear prolongation, the
               Hellmann-Feynman face gradient
  mg           the geometric-multigrid V(2,2) preconditioner T
  lobpcg       block LOBPCG following the algorithm of Section 2.2 with soft
               locking (Section 2.3)

Parity status: every function is pinned by a test in tests/ against the
closed form, brute-force dense eigensolves, algebraic identities or textbook
multigrid theory, except the V-cycle's exact definition beyond its
symmetry, positivity and two-grid error-propagation formula (the paper does
not define the multigrid it uses; the definition here is a reading).
"""
