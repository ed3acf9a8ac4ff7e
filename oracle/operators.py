"""Oracle: the ADR matrices and the standard Helmholtz matrix.  TEST INFRASTRUCTURE ONLY.

Row j of A_beta (eq. ADR discretized as in Sec. 2.2-2.3, blended as in eq. precADRup):

    (A_beta a)_j = sum_k (a_{j-e_k} - 2 a_j + a_{j+e_k}) / h^2
                   - 2 i w sum_k g_k,j (D_k^beta a)_j
                   - i w L_j avg(a)_j
                   + c_j a_j

* D_k^beta = (1-beta) D^2up + beta D^1up along axis k.  For g_k >= 0 the backward
  formulas of eq. londUpwindDiff, (3a_j - 4a_{j-1} + a_{j-2})/(2h) and (a_j-a_{j-1})/h;
  for g_k < 0 the forward mirror images.  H_2up = A_0, H_1up = A_1.
* Near the source (Chebyshev distance <= 1 node from it) every D_k is the central
  difference of eq. londDiff, whatever beta (Sec. 2.2).
* central=True gives H_cen (eq. ADRLinSystemCentral): D_k is the central difference of
  eq. londDiff at every node that has both neighbours along axis k; on the two face
  nodes of the axis, where it would need a node outside, the upwind operators (and
  their fallbacks, below) replace it, as Sec. 2.2.1 prescribes.
* Where an upwind stencil would leave the grid (Sec. 2.2.1 says it should not for an
  interior source; this fixes what happens when it does): one node short -> both
  orders use the first-order upwind formula; two nodes short (face node, g pointing
  inwards) -> the inward one-sided formulas of the same orders.
* avg(a)_j = (1/2d) sum_k (a_{j+e_k} + a_{j-e_k}) inside (the averaging mass of
  Sec. 2.3, taken isotropically), avg(a)_j = a_j on every boundary node.
* Faces: the Laplacian uses a ghost node from the Neumann condition for u rewritten for
  a, eq. BCADR read as n.grad a - i w (n.grad tau) a = 0: on the low face of axis k
  a_{-1} = a_1 - 2 h i w g_k a_0, on the high face a_n = a_{n-2} + 2 h i w g_k a_{n-1}.

Arrays use NumPy axis order (last axis = x); ``g`` is a list with one array per axis.
"""
import numpy as np
import scipy.sparse as sp


def _node_indices(shape):
    return np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")


def _advection_weights(mode, beta, h):
    """Weights {offset: w} of D^beta for one mode; offsets along the axis."""
    b2 = {0: 3.0 / (2 * h), -1: -4.0 / (2 * h), -2: 1.0 / (2 * h)}
    b1 = {0: 1.0 / h, -1: -1.0 / h}
    f2 = {0: -3.0 / (2 * h), 1: 4.0 / (2 * h), 2: -1.0 / (2 * h)}
    f1 = {0: -1.0 / h, 1: 1.0 / h}
    cen = {-1: -1.0 / (2 * h), 1: 1.0 / (2 * h)}

    def blend(second, first):
        out = {}
        for o, w in second.items():
            out[o] = out.get(o, 0.0) + (1.0 - beta) * w
        for o, w in first.items():
            out[o] = out.get(o, 0.0) + beta * w
        return out

    if mode == "B2":
        return blend(b2, b1)
    if mode == "F2":
        return blend(f2, f1)
    if mode == "B1":
        return dict(b1)
    if mode == "F1":
        return dict(f1)
    if mode == "C":
        return dict(cen)
    raise ValueError(mode)


def advection_modes(g_axis, axis, shape, src, central=False):
    """Per-node stencil choice along one axis: array of mode strings."""
    idx = _node_indices(shape)
    i = idx[axis]
    n = shape[axis]
    backward = g_axis >= 0.0
    mode = np.empty(shape, dtype=object)
    mode[backward & (i >= 2)] = "B2"
    mode[backward & (i == 1)] = "B1"
    mode[backward & (i == 0)] = "F2"
    fwd = ~backward
    mode[fwd & (i <= n - 3)] = "F2"
    mode[fwd & (i == n - 2)] = "F1"
    mode[fwd & (i == n - 1)] = "B2"
    if central:
        mode[(i >= 1) & (i <= n - 2)] = "C"
    if src is not None:
        cheb = np.max(np.stack([np.abs(idx[a] - src[a]) for a in range(len(shape))]), axis=0)
        mode[cheb <= 1] = "C"
    return mode


def adr_stencil(g, L, c, h, omega, beta, src=None, central=False):
    """Per-node stencil of A_beta as a dict {offset tuple: complex array}.

    Offsets are NumPy-axis-ordered tuples; entries that would reach outside the grid are
    checked to be exactly zero."""
    L = np.asarray(L, dtype=np.float64)
    c = np.asarray(c, dtype=np.complex128)
    shape = L.shape
    d = len(shape)
    idx = _node_indices(shape)
    zero = (0,) * d
    st = {zero: np.zeros(shape, dtype=np.complex128)}

    def off(axis, o):
        t = [0] * d
        t[axis] = o
        return tuple(t)

    def acc(key, val):
        if key not in st:
            st[key] = np.zeros(shape, dtype=np.complex128)
        st[key] += val

    on_face = np.zeros(shape, dtype=bool)
    for a in range(d):
        on_face |= (idx[a] == 0) | (idx[a] == shape[a] - 1)

    iw = 1j * omega
    for a in range(d):
        i = idx[a]
        n = shape[a]
        ga = np.asarray(g[a], dtype=np.float64)
        low = i == 0
        high = i == n - 1
        inner = ~(low | high)
        # Laplacian, with the ghost-node Robin rows on the faces.
        acc(off(a, -1), np.where(inner, 1.0 / h**2, 0.0) + np.where(high, 2.0 / h**2, 0.0))
        acc(off(a, +1), np.where(inner, 1.0 / h**2, 0.0) + np.where(low, 2.0 / h**2, 0.0))
        acc(zero, -2.0 / h**2 + np.where(low, -2.0 * iw * ga / h, 0.0) + np.where(high, 2.0 * iw * ga / h, 0.0))
        # Advection -2 i w g_k D_k^beta.
        modes = advection_modes(ga, a, shape, src, central)
        for m in ("B2", "B1", "F2", "F1", "C"):
            sel = modes == m
            if not np.any(sel):
                continue
            for o, w in _advection_weights(m, beta, h).items():
                acc(off(a, o), np.where(sel, -2.0 * iw * ga * w, 0.0))
        # Averaging mass -i w L avg(a): inner nodes only (boundary handled below).
        for o in (-1, 1):
            acc(off(a, o), np.where(on_face, 0.0, -iw * L / (2 * d)))
    st[zero] += np.where(on_face, -iw * L, 0.0)
    st[zero] += c

    # Entries pointing outside the grid must vanish.
    for key, val in st.items():
        for a in range(d):
            if key[a] != 0:
                i = idx[a] + key[a]
                outside = (i < 0) | (i >= shape[a])
                if np.any(val[outside] != 0):
                    raise AssertionError(f"stencil offset {key} reaches outside the grid")
    return st


def stencil_to_csr(st, shape):
    """Assemble a per-node stencil dict into a CSR matrix (row = flattened node)."""
    d = len(shape)
    idx = _node_indices(shape)
    N = int(np.prod(shape))
    rows, cols, vals = [], [], []
    flat = np.arange(N).reshape(shape)
    for key, val in st.items():
        inside = np.ones(shape, dtype=bool)
        nb = []
        for a in range(d):
            i = idx[a] + key[a]
            inside &= (i >= 0) & (i < shape[a])
            nb.append(i)
        sel = inside & (val != 0)
        r = flat[sel]
        cidx = np.ravel_multi_index(tuple(x[sel] for x in nb), shape)
        rows.append(r)
        cols.append(cidx)
        vals.append(val[sel])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    A.sum_duplicates()
    return A


def assemble_adr(g, L, c, h, omega, beta, src=None, central=False):
    """A_beta (or, with central=True, H_cen; beta then only matters on face nodes) as a
    CSR matrix (complex128)."""
    st = adr_stencil(g, L, c, h, omega, beta, src, central)
    return stencil_to_csr(st, np.asarray(L).shape)


def helmholtz_1d_laplacian(n, h):
    """1D second difference with the Neumann ghost u_{-1} = u_1, u_n = u_{n-2}."""
    main = np.full(n, -2.0)
    up = np.ones(n - 1)
    lo = np.ones(n - 1)
    up[0] = 2.0
    lo[-1] = 2.0
    return sp.diags([lo, main, up], [-1, 0, 1], format="csr") / (h * h)


def assemble_helmholtz(kappa2, gamma, h, omega):
    """Standard second-order Helmholtz matrix H (eq. HelmholtzLinSystem) with the
    absorbing term of Sec. 1:  Lap_h + diag(w^2 kappa^2 - i w gamma kappa^2).
    Built as a Kronecker sum of 1D matrices, independently of ``assemble_adr``."""
    kappa2 = np.asarray(kappa2, dtype=np.float64)
    shape = kappa2.shape
    d = len(shape)
    N = kappa2.size
    lap = sp.csr_matrix((N, N), dtype=np.float64)
    for a in range(d):
        mats = [sp.identity(n, format="csr") for n in shape]
        mats[a] = helmholtz_1d_laplacian(shape[a], h)
        term = mats[0]
        for m in mats[1:]:
            term = sp.kron(term, m, format="csr")
        lap = lap + term
    gam = np.zeros_like(kappa2) if gamma is None else np.asarray(gamma, dtype=np.float64)
    diag = omega * omega * kappa2 - 1j * omega * gam * kappa2
    return (lap.astype(np.complex128) + sp.diags(diag.ravel())).tocsr()
