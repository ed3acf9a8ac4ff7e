"""Oracle: geometric multigrid on the ADR preconditioner.  TEST INFRASTRUCTURE ONLY.

Paper, Sec. 3: relaxation plus coarse-grid correction; the coarse operator is the
Galerkin product A_c = P^T A P (eq. coarseGridMatrix) with P the bi/trilinear
interpolation (Sec. 3.1); the two-grid cycle (Alg. TwoCycle) applied recursively is the
V-cycle.  Relaxation (Sec. 3.1, Sec. 4.2) on level l uses l+1 pre- and post-relaxations:
* damped Jacobi  x <- x + w_J D^{-1} (b - A x)  per sweep (Sec. 3.1), used on the
  finest level where it is a smoother;
* Jacobi-preconditioned GMRES (the paper's relaxation, Sec. 4.2): nu steps of GMRES
  on A D^{-1} started from the current residual, i.e. x <- x + D^{-1} V y with y the
  least-squares minimizer of ||b - A(x + D^{-1} V y)|| over the Krylov space of
  A D^{-1} and r.  It is used on the coarse Galerkin levels, which are indefinite
  enough that damped Jacobi diverges there.
The coarsest system is solved exactly (dense LU); this replaces the paper's ten inexact
GMRES steps.

The Krylov cycle (Sec. 3.1, Alg. KrylovCycle) replaces the recursive coarse solve of
every level that is not the coarsest by flexible GMRES with two steps, started from
zero and preconditioned by the Krylov cycle one level down.  The second step is left
out when the first one already reduced the coarse residual below a threshold times its
initial norm (0.1, Sec. 4.2.2, following Notay and Vassilevski).

Grids are nodal with n_c = (n_f - 1)/2 + 1 nodes per axis; coarse node I coincides with
fine node 2I.  P is real, so P^T = P^H (complex data).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def prolongation_1d(n_fine):
    """Linear interpolation, n_fine x n_coarse: P[2I, I] = 1, P[2I +- 1, I] = 1/2."""
    if (n_fine - 1) % 2:
        raise ValueError("n_fine - 1 must be even")
    n_c = (n_fine - 1) // 2 + 1
    rows, cols, vals = [], [], []
    for I in range(n_c):
        rows.append(2 * I)
        cols.append(I)
        vals.append(1.0)
        for o in (-1, 1):
            f = 2 * I + o
            if 0 <= f < n_fine:
                rows.append(f)
                cols.append(I)
                vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n_fine, n_c))


def prolongation(shape):
    """Tensor-product (bi/tri)linear interpolation for a C-ordered grid of ``shape``."""
    P = None
    for n in shape:
        p = prolongation_1d(n)
        P = p if P is None else sp.kron(P, p, format="csr")
    return P.tocsr()


def coarse_shape(shape):
    return tuple((n - 1) // 2 + 1 for n in shape)


class Hierarchy:
    """Levels 0..L-1 (level 0 = finest): operators A[l], interpolations P[l] (level l+1 ->
    l), Jacobi diagonals, sweep counts and a dense LU of the coarsest operator."""

    def __init__(self, A_fine, shape, levels, nu=None, jacobi_weight=0.8, smoothers=None):
        self.shapes = [tuple(shape)]
        self.A = [A_fine.tocsr()]
        self.P = []
        for _ in range(levels - 1):
            s = self.shapes[-1]
            P = prolongation(s)
            Ac = (P.T @ self.A[-1] @ P).tocsr()
            Ac.sum_duplicates()
            self.P.append(P)
            self.A.append(Ac)
            self.shapes.append(coarse_shape(s))
        self.levels = levels
        # Level l (0-based) gets l+2 relaxations: 2 on the finest, 3 on the next, ...
        self.nu = list(nu) if nu is not None else [l + 2 for l in range(levels)]
        self.w = jacobi_weight
        # Default: Jacobi on the finest level, GMRES relaxation on the coarse levels.
        self.smoothers = list(smoothers) if smoothers is not None else \
            ["jacobi"] + ["gmres"] * (levels - 1)
        self.dinv = [1.0 / A.diagonal() for A in self.A]
        self.coarse_lu = sla.lu_factor(self.A[-1].toarray())

    def jacobi(self, l, x, b, sweeps):
        A, dinv, w = self.A[l], self.dinv[l], self.w
        for _ in range(sweeps):
            x = x + w * dinv * (b - A @ x)
        return x

    def gmres_relax(self, l, x, b, steps):
        """``steps`` Arnoldi steps (modified Gram-Schmidt) on A D^{-1} from r = b - A x,
        then the small least-squares solve; returns x + D^{-1} V y."""
        A, dinv = self.A[l], self.dinv[l]
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta == 0.0:
            return x
        V = [r / beta]
        H = np.zeros((steps + 1, steps), dtype=np.complex128)
        k = 0
        for j in range(steps):
            w = A @ (dinv * V[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            if H[j + 1, j] == 0.0:
                break
            V.append(w / H[j + 1, j])
        rhs = np.zeros(k + 1, dtype=np.complex128)
        rhs[0] = beta
        y = np.linalg.lstsq(H[:k + 1, :k], rhs, rcond=None)[0]
        return x + dinv * (np.array(V[:k]).T @ y)

    def relax(self, l, x, b):
        if self.smoothers[l] == "jacobi":
            return self.jacobi(l, x, b, self.nu[l])
        if self.smoothers[l] == "gmres":
            return self.gmres_relax(l, x, b, self.nu[l])
        raise ValueError(self.smoothers[l])

    def kcycle(self, b, l=0, threshold=0.1, kmax=0):
        """One Krylov cycle from a zero initial guess on level l: x ~ A_l^{-1} b.
        ``self.kcalls[l]`` counts the cycles entered on level l.  ``kmax`` > 0 keeps the
        flexible-GMRES coarse solve for coarse levels 1..kmax only; deeper coarse problems
        are solved by the same cycle directly, as in the V-cycle."""
        if not hasattr(self, "kcalls"):
            self.kcalls = [0] * self.levels
        self.kcalls[l] += 1
        if l == self.levels - 1:
            return sla.lu_solve(self.coarse_lu, b)
        x = np.zeros_like(b)
        x = self.relax(l, x, b)
        r = b - self.A[l] @ x
        rc = self.P[l].T @ r
        if l + 1 == self.levels - 1:
            ec = sla.lu_solve(self.coarse_lu, rc)
        elif kmax <= 0 or l + 1 <= kmax:
            ec = self.coarse_fgmres(l + 1, rc, threshold, kmax)
        else:
            ec = self.kcycle(rc, l + 1, threshold, kmax)
        x = x + self.P[l] @ ec
        x = self.relax(l, x, b)
        return x

    def coarse_fgmres(self, l, r, threshold, kmax=0):
        """Flexible GMRES(2) on A_l e = r from e = 0, preconditioned by the Krylov cycle
        on level l; one step only if its residual is <= threshold * ||r||."""
        A = self.A[l]
        beta = np.linalg.norm(r)
        if beta == 0.0:
            return np.zeros_like(r)
        V = [r / beta]
        Z = []
        H = np.zeros((3, 2), dtype=np.complex128)
        k = 0
        for j in range(2):
            Z.append(self.kcycle(V[j], l, threshold, kmax) if kmax > 0 else self.kcycle(V[j], l, threshold))
            w = A @ Z[j]
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            rhs = np.zeros(k + 1, dtype=np.complex128)
            rhs[0] = beta
            y, *_ = np.linalg.lstsq(H[:k + 1, :k], rhs, rcond=None)
            res = np.linalg.norm(rhs - H[:k + 1, :k] @ y)
            if j == 0 and (res <= threshold * beta or H[1, 0] == 0.0):
                break
            if j == 0:
                V.append(w / H[1, 0])
        return np.array(Z[:k]).T @ y

    def vcycle(self, b, l=0):
        """One V-cycle from a zero initial guess on level l: returns x ~ A_l^{-1} b."""
        if l == self.levels - 1:
            return sla.lu_solve(self.coarse_lu, b)
        x = np.zeros_like(b)
        x = self.relax(l, x, b)
        r = b - self.A[l] @ x
        rc = self.P[l].T @ r
        ec = self.vcycle(rc, l + 1)
        x = x + self.P[l] @ ec
        x = self.relax(l, x, b)
        return x
