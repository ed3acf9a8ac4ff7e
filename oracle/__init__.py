"""Plain FP64 CPU oracle for the ADR-amplitude solve of Treister & Haber (arXiv:1712.06091).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its Python
binding, the solve benchmark's timed leg) may import, call or link this package; only
the test-suite, the smoke check and the benchmark's CPU-baseline leg do.  It shares no
code with the GPU path and imports nothing from it: inputs (kappa^2, tau, gamma, source
node, right-hand side) are passed in as plain NumPy arrays.

What it computes, in the paper's order:

* ``coefficients``  -- grad(tau), Laplacian(tau) and the reaction term from a factored
  travel time (Sec. 2.1, eq. travel_time_coeff; reaction from eq. ADR with the
  absorbing term of Sec. 1).
* ``operators``     -- the ADR matrices A_beta = (1-beta) H_2up + beta H_1up
  (Sec. 2.2, eqs. londDiff / londUpwindDiff, the averaging mass of Sec. 2.3, the
  boundary condition eq. BCADR, the preconditioner eq. precADRup) and, written
  independently, the standard Helmholtz matrix H (eq. HelmholtzLinSystem).
* ``multigrid``     -- bilinear / trilinear prolongation, Galerkin coarse operators
  (eq. coarseGridMatrix), damped Jacobi and the V-cycle (Alg. TwoCycle applied
  recursively, Sec. 3).
* ``krylov``        -- restarted flexible GMRES (Sec. 3.1, Sec. 4.2).
* ``solve``         -- direct and iterative solves of H_2up a = q_hat, the wavefield
  u = a exp(-i w tau) (eq. new_u), the adjoint solve and the kappa^2 gradient.
* ``closed_form``   -- constant-medium Green's functions used as pins (Sec. 1).

Every function is FP64 (complex128 for complex data).
"""
