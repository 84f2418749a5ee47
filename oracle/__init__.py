"""CPU FP64 oracle for the implicit-time immersed-boundary multigrid solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the GPU library: every operator
here is assembled as an explicit scipy.sparse matrix straight from the
paper's definitions, and the algorithms (box relaxation, V-cycle, FGMRES,
time step) follow the paper's steps in its order and notation.

Paper: Guy, Philip, Griffith, "Geometric multigrid for an implicit-time
immersed boundary method" (arXiv 1311.5614).

Module map
  mac        MAC-grid Laplacian, gradient, divergence, grid transfers (Sec. 2.2, 3.1)
  ib         regularised delta, spreading/interpolation, fibre operator (Sec. 2.2)
  system     implicit-step operator and hybrid coarse operators (Sec. 2.3, 3, 3.2, 8)
  smoother   (big-)box relaxation (Sec. 5, 6)
  mg         V-cycle, Algorithm 1, with a bordered coarsest solve (Sec. 3)
  krylov     right-preconditioned flexible GMRES (Sec. 3.3)
  step       one implicit IB time step (Sec. 2.3.2 with the unsteady form of Sec. 8)
  stokes_fft spectral solve of the periodic MAC Stokes problem (test pin)
  dtexp      explicit stability limit, Sec. 4.1, via Lanczos

Pins (the tests under tests/oracle_*) tie each function to closed forms,
invariants, brute force on tiny inputs and a spectral special case.  The one
result without a hard pin, the MG iteration-matrix spectral radius for the
periodic problem, is reported as "parity unpinned" in the tests that touch it.
"""
