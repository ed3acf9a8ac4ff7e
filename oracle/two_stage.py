"""Oracle: the ADR system with central advection and its two-stage solve.
TEST INFRASTRUCTURE ONLY.

Sec. 3.2, Alg. ADRlong, with the settings of Sec. 4.2:
* H_cen (eq. ADRLinSystemCentral) is the ADR operator with the central advection of
  eq. londDiff (``operators.assemble_adr(..., central=True)``, beta = 0 on the faces).
* Stage 1: a_1up, a low-accuracy solution of H_1up a = q_hat (eq. 1up): flexible
  GMRES(5) preconditioned by the Krylov cycle on H_1up itself, at most 5 cycles,
  stopping earlier once the relative residual of eq. 1up is 1e-2.
* Stage 2: with M = diag(exp(-i w tau)) and u_1up = M a_1up, flexible GMRES on the
  rescaled system M H_cen M^{-1} u = q (eq. ADRcenRescaled) started from u_1up,
  preconditioned by a multigrid cycle on the shifted operator
  H_s^cen = M H_cen M^{-1} - i w^2 alpha diag(kappa^2), alpha = 0.2, whose coarse
  operators are its own Galerkin products (the coarsening acts on u, not on a).
* Result: u, and a = M^{-1} u.
"""
import numpy as np
import scipy.sparse as sp

from . import coefficients, krylov, multigrid, operators, solve


class TwoStageProblem:
    """H_1up, H_cen and the rescaled stage-2 matrices for one source."""

    def __init__(self, kappa2, tau, gamma, h, omega, src, alpha=0.2, factored=True):
        self.kappa2 = np.asarray(kappa2, dtype=np.float64)
        self.tau = np.asarray(tau, dtype=np.float64)
        self.shape = self.tau.shape
        self.h, self.omega, self.src, self.alpha = h, omega, tuple(src), alpha
        g, L, c = coefficients.adr_coefficients(self.tau, self.kappa2, gamma, h, omega,
                                                src=self.src if factored else None)
        self.H1up = operators.assemble_adr(g, L, c, h, omega, 1.0, src=self.src)
        self.Hcen = operators.assemble_adr(g, L, c, h, omega, 0.0, src=self.src, central=True)
        m = np.exp(-1j * omega * self.tau.ravel())          # diagonal of M
        self.m = m
        self.B = (sp.diags(m) @ self.Hcen @ sp.diags(1.0 / m)).tocsr()
        self.Bs = (self.B - 1j * omega * omega * alpha * sp.diags(self.kappa2.ravel())).tocsr()

    def stage1(self, qhat, levels=None, tol=1e-2, maxit=5, threshold=0.1):
        if levels is None:
            levels = solve.default_levels(self.shape)
        hier = multigrid.Hierarchy(self.H1up, self.shape, levels)
        return krylov.fgmres(lambda v: self.H1up @ v, qhat, precond=lambda v: hier.kcycle(v, threshold=threshold),
                             restart=5, tol=tol, maxit=maxit)

    def stage2(self, q, u0, levels=None, tol=1e-10, maxit=500, cycle="k", threshold=0.1):
        if levels is None:
            levels = solve.default_levels(self.shape)
        hier = multigrid.Hierarchy(self.Bs, self.shape, levels)
        if cycle == "k":
            precond = lambda v: hier.kcycle(v, threshold=threshold)
        else:
            precond = hier.vcycle
        return krylov.fgmres(lambda v: self.B @ v, q, precond=precond, x0=u0, restart=5, tol=tol, maxit=maxit)


def two_stage_solve(prob, q, tol=1e-10, maxit=500, stage1_tol=1e-2, stage1_maxit=5, cycle="k", levels=None):
    """Alg. ADRlong.  q is the Helmholtz right-hand side; returns (u, a, info1, info2)."""
    q = np.asarray(q, dtype=np.complex128).ravel()
    qhat = q / prob.m                                       # q_hat = M^{-1} q = q exp(i w tau)
    a1, info1 = prob.stage1(qhat, levels=levels, tol=stage1_tol, maxit=stage1_maxit)
    u1 = prob.m * a1                                        # u_1up = M a_1up
    u, info2 = prob.stage2(q, u1, levels=levels, tol=tol, maxit=maxit, cycle=cycle)
    a = u / prob.m
    return u.reshape(prob.shape), a.reshape(prob.shape), info1, info2
