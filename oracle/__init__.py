"""CPU oracle for the 2D Lippmann-Schwinger solver (test infrastructure only).

This package is test infrastructure.  Only the test suite, the smoke check in
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (the HIP library and its Python binding) never
imports, calls or links anything here, and nothing here imports the product.

Contents (each function cites the passage of the paper it follows):

* ``special``  -- the Helmholtz Green's function G = (i/4) H0^(1)(kappa r) via
  scipy, and the exact singular self-cell integral for one-point (p = 1) cells.
* ``lsop``     -- the discretised volume operator V (dense, by its definition),
  the same product through a zero-padded FFT convolution, the LS operator
  A = I + s kappa^2 diag(q) V and the plane-wave right-hand side.
* ``gmres``    -- restarted GMRES (modified Gram-Schmidt Arnoldi, Givens
  rotations), optionally right-preconditioned.
* ``hodlr``    -- the fixed-rank HODLR approximation of A built with partially
  pivoted ACA and its recursive Sherman-Morrison-Woodbury inverse.
* ``mie``      -- the Bessel-series (Mie) solution for a constant-contrast disc.

Every routine is plain, unblocked FP64 (complex128) numpy/scipy code.
"""
