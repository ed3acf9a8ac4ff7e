"""Oracle: solves of H_2up a = q_hat, the wavefield, the adjoint and the kappa^2 gradient.
TEST INFRASTRUCTURE ONLY.

* q_hat = q exp(i w tau) (eq. ADR); a point source is q = e_src / h^d (Sec. 4.1).
* u = a exp(-i w tau) (eq. new_u).
* Outer solve: flexible GMRES(m) on H_2up, preconditioned by a V-cycle on
  A_beta = (1-beta) H_2up + beta H_1up, beta = 0.25 (eq. precADRup, Sec. 4.2).
* Adjoint (not in the paper): for J = 1/2 sum_s ||R u_s - d_s||^2 at fixed tau,
  dH_2up/dkappa2_j = c'_j e_j e_j^T with c'_j = w^2 - i w gamma_j (numerical reaction)
  or -i w gamma_j (eikonal reaction), so with
  lambda = H_2up^{-H} M^H R^T (R M a - d), M = diag(exp(-i w tau)),
  dJ/dkappa2_j = -Re(conj(lambda_j) c'_j a_j).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import coefficients, krylov, multigrid, operators


def point_source_rhs(shape, src, h):
    q = np.zeros(shape, dtype=np.complex128)
    q[tuple(src)] = 1.0 / h ** len(shape)
    return q


def rhs_hat(q, tau, omega):
    return np.asarray(q, dtype=np.complex128) * np.exp(1j * omega * np.asarray(tau))


def wavefield(a, tau, omega):
    return np.asarray(a) * np.exp(-1j * omega * np.asarray(tau))


class Problem:
    """The discrete ADR problem for one source: coefficients and the two operators."""

    def __init__(self, kappa2, tau, gamma, h, omega, src, beta=0.25, factored=True, reaction="numerical"):
        self.shape = np.asarray(tau).shape
        self.h, self.omega, self.src, self.beta = h, omega, tuple(src), beta
        self.reaction = reaction
        self.kappa2 = np.asarray(kappa2, dtype=np.float64)
        self.tau = np.asarray(tau, dtype=np.float64)
        self.gamma = None if gamma is None else np.asarray(gamma, dtype=np.float64)
        fsrc = self.src if factored else None
        self.g, self.L, self.c = coefficients.adr_coefficients(
            self.tau, self.kappa2, self.gamma, h, omega, src=fsrc, form=reaction)
        self.H2up = operators.assemble_adr(self.g, self.L, self.c, h, omega, 0.0, src=self.src)
        self.Abeta = operators.assemble_adr(self.g, self.L, self.c, h, omega, beta, src=self.src)

    def hierarchy(self, levels=None, nu=None, jacobi_weight=0.8, smoothers=None):
        if levels is None:
            levels = default_levels(self.shape)
        return multigrid.Hierarchy(self.Abeta, self.shape, levels, nu=nu,
                                   jacobi_weight=jacobi_weight, smoothers=smoothers)


def default_levels(shape, coarsest_max=729, min_coarse=5):
    """Halve every axis while n-1 is even, the coarse grid keeps >= min_coarse nodes per
    axis and the current grid has more than coarsest_max nodes."""
    levels = 1
    s = tuple(shape)
    while int(np.prod(s)) > coarsest_max and all((n - 1) % 2 == 0 for n in s) \
            and all((n - 1) // 2 + 1 >= min_coarse for n in s):
        s = tuple((n - 1) // 2 + 1 for n in s)
        levels += 1
    return levels


def direct_solve(A, b):
    """Dense LU for small systems, sparse LU otherwise."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    if A.shape[0] <= 5000:
        return sla.solve(A.toarray(), b)
    return spla.splu(A.tocsc()).solve(b)


def iterative_solve(prob, qhat, levels=None, tol=1e-10, maxit=500, restart=5, nu=None,
                    jacobi_weight=0.8, smoothers=None, cycle="v", threshold=0.1, kmax=0):
    """FGMRES(restart) on H_2up preconditioned by one V-cycle (cycle="v") or one Krylov
    cycle (cycle="k") on A_beta per step."""
    hier = prob.hierarchy(levels, nu=nu, jacobi_weight=jacobi_weight, smoothers=smoothers)
    if cycle == "v":
        precond = hier.vcycle
    elif cycle == "k":
        precond = lambda v: hier.kcycle(v, threshold=threshold, kmax=kmax)
    else:
        raise ValueError(cycle)
    x, info = krylov.fgmres(lambda v: prob.H2up @ v, qhat.ravel(), precond=precond,
                            restart=restart, tol=tol, maxit=maxit)
    return x.reshape(prob.shape), info


def adjoint_gradient(prob, a, receivers, d_obs, solve=direct_solve):
    """Misfit J = 1/2 ||R u - d||^2 for one source and its gradient w.r.t. kappa^2.

    ``receivers`` is a tuple of index arrays (NumPy axis order) selecting u at receiver
    nodes (R is a 0/1 sampling operator)."""
    u = wavefield(a, prob.tau, prob.omega)
    res = u[receivers] - d_obs
    J = 0.5 * float(np.sum(np.abs(res) ** 2))
    rhs = np.zeros(prob.shape, dtype=np.complex128)
    np.add.at(rhs, receivers, res)
    rhs = np.conj(np.exp(-1j * prob.omega * prob.tau)) * rhs   # M^H R^T r
    lam = solve(prob.H2up.conj().T.tocsr(), rhs.ravel()).reshape(prob.shape)
    dc = coefficients.reaction_derivative(prob.gamma, prob.omega, prob.shape, prob.reaction)
    grad = -np.real(np.conj(lam) * dc * a)
    return J, grad, lam
