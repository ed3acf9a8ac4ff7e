"""Oracle: restarted flexible GMRES.  TEST INFRASTRUCTURE ONLY.

Paper: Sec. 3.1 and Sec. 4.2 -- flexible GMRES(m) (Saad 1993) with a multigrid cycle as
the (right) preconditioner, zero initial guess, stopped on the relative residual.
Here the stopping test is the true residual ||b - A x|| / ||b||, evaluated at every
restart and at exit; inside a cycle the Givens-rotated Arnoldi estimate decides when to
leave early.  Orthogonalization is modified Gram-Schmidt with the Hermitian inner
product <u, v> = sum conj(u) v.
"""
import numpy as np


def fgmres(matvec, b, precond=None, x0=None, restart=5, tol=1e-6, maxit=500):
    """Solve A x = b.  Returns (x, info) where info holds the outer iteration count, the
    true relative residual and the per-iteration estimate history."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    M = (lambda v: v) if precond is None else precond
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), {"iters": 0, "relres": 0.0, "history": []}
    history = []
    iters = 0
    r = b - matvec(x)
    relres = np.linalg.norm(r) / bnorm
    while relres > tol and iters < maxit:
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, n), dtype=np.complex128)
        Z = np.zeros((restart, n), dtype=np.complex128)
        Hm = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        s = np.zeros(restart + 1, dtype=np.complex128)
        s[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            Z[j] = M(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                Hm[i, j] = np.vdot(V[i], w)
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] != 0.0:
                V[j + 1] = w / Hm[j + 1, j]
            # Apply the earlier rotations to the new column, then form a new one.
            for i in range(j):
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -np.conj(sn[i]) * Hm[i, j] + np.conj(cs[i]) * Hm[i + 1, j]
                Hm[i, j] = t
            a, bb = Hm[j, j], Hm[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if a == 0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                # G = [[c, s], [-conj(s), c]] with real c zeroes the subdiagonal.
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(bb) / den
            Hm[j, j] = cs[j] * a + sn[j] * bb
            Hm[j + 1, j] = 0.0
            s[j + 1] = -np.conj(sn[j]) * s[j]
            s[j] = cs[j] * s[j]
            k = j + 1
            iters += 1
            history.append(abs(s[j + 1]) / bnorm)
            if abs(s[j + 1]) / bnorm <= tol or iters >= maxit:
                break
        y = np.linalg.solve(np.triu(Hm[:k, :k]), s[:k])
        x = x + Z[:k].T @ y
        r = b - matvec(x)
        relres = np.linalg.norm(r) / bnorm
    return x, {"iters": iters, "relres": relres, "history": history}
