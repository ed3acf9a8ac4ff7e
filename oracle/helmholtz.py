"""Oracle: the standard Helmholtz system and the shifted-Laplacian preconditioner.
TEST INFRASTRUCTURE ONLY.

* The standard second-order discretization H u = q (Sec. 2, eq. HelmholtzLinSystem):
  H = Lap_h + diag(w^2 kappa^2 - i w gamma kappa^2), the absorbing term of Sec. 1
  included, with the ghost-node Neumann faces of the ADR operator (Sec. 2.2).  H is
  assembled by ``operators.assemble_helmholtz`` as a Kronecker sum of 1D matrices,
  independently of the ADR stencil.
* The shifted operator H_s = H - i w^2 alpha diag(kappa^2), alpha > 0 (Sec. 3.1,
  eq. shift): the preconditioner, approximately inverted by one multigrid cycle with
  Galerkin coarse operators P^T H_s P, inside flexible GMRES on H.  The paper's
  Helmholtz runs use alpha = 0.2 (Sec. 4.2).
* The wavefield is u itself (tau = 0: no phase factor).
"""
import numpy as np
import scipy.sparse as sp

from . import krylov, multigrid, operators, solve


class HelmholtzProblem:
    """H and H_s for one medium."""

    def __init__(self, kappa2, gamma, h, omega, alpha=0.2):
        self.kappa2 = np.asarray(kappa2, dtype=np.float64)
        self.shape = self.kappa2.shape
        self.gamma = None if gamma is None else np.asarray(gamma, dtype=np.float64)
        self.h, self.omega, self.alpha = h, omega, alpha
        self.H = operators.assemble_helmholtz(self.kappa2, self.gamma, h, omega)
        shift = -1j * omega * omega * alpha * self.kappa2.ravel()
        self.Hs = (self.H + sp.diags(shift)).tocsr()

    def hierarchy(self, levels=None, nu=None, jacobi_weight=0.8, smoothers=None):
        if levels is None:
            levels = solve.default_levels(self.shape)
        return multigrid.Hierarchy(self.Hs, self.shape, levels, nu=nu,
                                   jacobi_weight=jacobi_weight, smoothers=smoothers)


def iterative_solve(prob, q, levels=None, tol=1e-10, maxit=500, restart=5, nu=None,
                    jacobi_weight=0.8, smoothers=None, cycle="v", threshold=0.1):
    """FGMRES(restart) on H preconditioned by one V-cycle (cycle="v") or one Krylov cycle
    (cycle="k") on H_s per step."""
    hier = prob.hierarchy(levels, nu=nu, jacobi_weight=jacobi_weight, smoothers=smoothers)
    if cycle == "v":
        precond = hier.vcycle
    elif cycle == "k":
        precond = lambda v: hier.kcycle(v, threshold=threshold)
    else:
        raise ValueError(cycle)
    x, info = krylov.fgmres(lambda v: prob.H @ v, np.asarray(q, dtype=np.complex128).ravel(),
                            precond=precond, restart=restart, tol=tol, maxit=maxit)
    return x.reshape(prob.shape), info
