"""FP64 CPU oracle for the dispersion-matching two-grid Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the HIP path is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never calls it, and it shares no code with the HIP library
(both take their inputs from the separate `synthetic` module).

Every function cites the passage of Stolk, "A two-grid method with dispersion
matching for finite-element Helmholtz problems" (arXiv 2509.17494) that it
follows.  Library primitives used as steps: scipy.sparse assembly, sparse LU
(splu), dense LAPACK solves, numpy eigenvalue routines.

Modules
  fem        GLL Lagrange Q_p space, exact 1-D reference matrices, assembly of
             a(u,v; Omega, Gamma_abs) (eq. bilin_form, Sec. 2-3.1)
  qsfem      QSFEM stencil, scaling and the quasi-FE coarse matrix (Sec. 3.2-3.3)
  transfer   Q_{p/2} interpolation prolongation and its adjoint (Sec. 4.2)
  smoother   complex-shifted DD smoother, Alg. 2 with the averaged update
  twogrid    Alg. 1, the preconditioner map and right-preconditioned GMRES
  lfa        toy 1-D LFA (Sec. 5), Bloch-wave symbols (Sec. 6.1)
  dispersion discrete dispersion of the fine FE scheme and the plain
             dispersion-matching fit of the 9-point family (parity unpinned
             beyond the invariants listed there)
  mlp        FP64 forward/backward of the coarse-stencil surrogate
"""
