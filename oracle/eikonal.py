"""Oracle: first-arrival travel time from the factored eikonal equation by fixed-point
sweeps.  TEST INFRASTRUCTURE ONLY.

Paper, Sec. 1, eq. factoredEikonal: with tau = tau0 * tau1 and tau0 = |x - x0|,
    |tau0 grad tau1 + tau1 grad tau0|^2 = kappa^2,
where grad tau0 = (x - x0)/|x - x0| is known; tau1(x0) = kappa(x0).  The paper computes
tau1 by factored fast marching and notes that fast sweeping or other iterative solvers of
the same equation can serve (Sec. 1).  This is the iterative form, written plainly: every
sweep recomputes each node's value from its neighbours' values of the previous sweep
(all nodes at once) and keeps the smaller of the old and the new value; the sweeps stop
when nothing changes.

Local update of node i (not the source), grid spacing h, r = tau0(x_i), p = grad tau0:
* per axis k, the neighbour j with the smaller tau (the minus side on ties) is the
  upwind one, unless its tau is still infinite; s_k = +1 for the neighbour at x - h e_k,
  -1 for x + h e_k; the first-order one-sided difference s_k (tau1_i - tau1_j)/h of tau1
  gives the k-th component of grad tau as A_k tau1_i + B_k, A_k = r s_k/h + p_k,
  B_k = -r s_k tau1_j/h;
* for a subset S of those axes (the others take d tau1/dx_k = 0: component p_k tau1_i),
  the larger root T of sum_{k in S} (A_k T + B_k)^2 + sum_{k not in S} (p_k T)^2 = kappa_i^2
  is admissible if it is positive and, on every axis in S, the gradient component points
  away from the upwind neighbour (s_k (A_k T + B_k) >= -1e-12 |T|) and r T >= tau_j;
* the candidate is r T from the largest admissible S, the smallest T among subsets of
  that size (dropping an axis is only a fallback);
* safeguard (a first arrival is Lipschitz with the local slowness): the candidate must
  not exceed min_j (tau_j + 1.1 h max(kappa_i, kappa_j)) over the 2d neighbours; if it
  does, or no subset is admissible, the candidate is the first-order Godunov update of
  the unfactored equation, sum over the u smallest per-axis upwind values t_k of
  (T - t_k)^2 = (h kappa_i)^2 with u grown while T exceeds the next value.

Arrays use NumPy axis order; ``src`` is a NumPy index tuple.
"""
import numpy as np

CAUSAL_EPS = 1e-12
LIPSCHITZ = 1.1


def _neighbour(a, axis, offset, fill):
    """a at the node offset by +-1 along `axis` (fill outside the grid)."""
    out = np.full_like(a, fill)
    dst = [slice(None)] * a.ndim
    srcs = [slice(None)] * a.ndim
    if offset > 0:
        dst[axis], srcs[axis] = slice(0, -1), slice(1, None)
    else:
        dst[axis], srcs[axis] = slice(1, None), slice(0, -1)
    out[tuple(dst)] = a[tuple(srcs)]
    return out


def sweep(tau, kappa2, h, src):
    """One sweep: the candidate of every node from `tau`, then min(old, candidate)."""
    shape = tau.shape
    d = tau.ndim
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    dx = [(grids[a] - src[a]) * h for a in range(d)]
    r = np.sqrt(sum(x * x for x in dx))
    at_src = r == 0.0
    r_safe = np.where(at_src, 1.0, r)
    p = [np.where(at_src, 0.0, x / r_safe) for x in dx]
    kap = np.sqrt(kappa2)
    tau1 = np.where(at_src, kap, tau / r_safe)

    A, B, tn, sd = [], [], [], []
    for a in range(d):
        tm, tp = _neighbour(tau, a, -1, np.inf), _neighbour(tau, a, +1, np.inf)
        t1m, t1p = _neighbour(tau1, a, -1, 0.0), _neighbour(tau1, a, +1, 0.0)
        minus = tm <= tp
        s = np.where(minus, 1.0, -1.0)
        t1n = np.where(minus, t1m, t1p)
        tn.append(np.where(minus, tm, tp))
        sd.append(s)
        A.append(r * s / h + p[a])
        with np.errstate(invalid="ignore"):
            B.append(np.where(np.isfinite(tn[-1]), -r * s * t1n / h, 0.0))

    best = np.full(shape, np.inf)
    best_size = np.zeros(shape, dtype=np.int64)
    for mask in range(1, 1 << d):
        S = [a for a in range(d) if mask >> a & 1]
        qa = sum(A[a] * A[a] if a in S else p[a] * p[a] for a in range(d))
        qb = sum(2.0 * A[a] * B[a] for a in S)
        qc = sum(B[a] * B[a] for a in S) - kappa2
        disc = qb * qb - 4.0 * qa * qc
        ok = (disc >= 0.0) & (qa > 0.0)
        with np.errstate(invalid="ignore", divide="ignore"):
            T = (-qb + np.sqrt(np.where(ok, disc, 0.0))) / (2.0 * qa)
        ok &= T > 0.0
        for a in S:
            ok &= np.isfinite(tn[a])
            ok &= sd[a] * (A[a] * T + B[a]) >= -CAUSAL_EPS * np.abs(T)
            ok &= r * T >= tn[a]
        take = ok & ((len(S) > best_size) | ((len(S) == best_size) & (T < best)))
        best = np.where(take, T, best)
        best_size = np.where(take, len(S), best_size)
    with np.errstate(invalid="ignore"):
        cand = np.where(np.isfinite(best), r * best, np.inf)

    # Safeguard: Lipschitz bound over the 2d neighbours, unfactored Godunov fallback.
    bound = np.full(shape, np.inf)
    for a in range(d):
        for o in (-1, 1):
            tj = _neighbour(tau, a, o, np.inf)
            kj = np.sqrt(_neighbour(kappa2, a, o, 0.0))
            bound = np.minimum(bound, tj + LIPSCHITZ * h * np.maximum(kap, kj))
    t_axis = np.sort(np.stack(tn), axis=0)
    f = h * kap
    tg = t_axis[0] + f
    grow = np.ones(shape, dtype=bool)
    for u in range(2, d + 1):
        grow &= tg > t_axis[u - 1]
        qa = float(u)
        qb = -2.0 * sum(t_axis[k] for k in range(u))
        qc = sum(t_axis[k] * t_axis[k] for k in range(u)) - f * f
        with np.errstate(invalid="ignore"):
            disc = qb * qb - 4.0 * qa * qc
            grow &= disc >= 0.0
            root = (-qb + np.sqrt(np.where(grow, disc, 0.0))) / (2.0 * qa)
        tg = np.where(grow, root, tg)
    fallback = ~np.isfinite(cand) | (cand > bound)
    cand = np.where(fallback, tg, cand)
    cand[tuple(src)] = 0.0
    return np.minimum(tau, cand)


def factored_eikonal(kappa2, h, src, max_sweeps=100000):
    """Fixed point of the sweeps from tau = 0 at the source and +inf elsewhere.
    Returns (tau, number of sweeps that changed some value)."""
    kappa2 = np.asarray(kappa2, dtype=np.float64)
    tau = np.full(kappa2.shape, np.inf)
    tau[tuple(src)] = 0.0
    for k in range(max_sweeps):
        new = sweep(tau, kappa2, h, tuple(src))
        if np.array_equal(new, tau):
            return tau, k
        tau = new
    raise RuntimeError("factored eikonal sweeps did not converge")
