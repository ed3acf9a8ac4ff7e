"""Helpers for the oracle pins: Dirichlet solves and manufactured solutions (test code)."""
import numpy as np
import scipy.sparse.linalg as spla


def boundary_mask(shape):
    d = len(shape)
    bnd = np.zeros(shape, dtype=bool)
    for a in range(d):
        sl = [slice(None)] * d
        sl[a] = 0
        bnd[tuple(sl)] = True
        sl[a] = -1
        bnd[tuple(sl)] = True
    return bnd


def solve_dirichlet(A, shape, rhs, boundary_values):
    """Solve the interior rows of A x = rhs with x fixed to ``boundary_values`` on faces."""
    B = boundary_mask(shape).ravel()
    I = ~B
    A = A.tocsr()
    bv = np.asarray(boundary_values, dtype=np.complex128).ravel()
    r = np.asarray(rhs, dtype=np.complex128).ravel()[I] - A[I][:, B] @ bv[B]
    xi = spla.splu(A[I][:, I].tocsc()).solve(r)
    x = bv.copy()
    x[I] = xi
    return x.reshape(shape)
