"""Oracle: ADR coefficients from a (factored) travel time.  TEST INFRASTRUCTURE ONLY.

Arrays are C-ordered NumPy arrays whose last axis is x (the fastest grid direction);
node j sits at position j*h along each axis.  ``src`` is the source node as a NumPy
index tuple in the same axis order (so ``src = (iz, iy, ix)`` in 3D).

Paper: Sec. 2.1, eq. (travel_time_coeff): with tau = tau0 * tau1 and tau0 = |x - x0|,
    grad tau = tau0 grad tau1 + tau1 grad tau0,
    lap  tau = tau1 lap tau0 + 2 grad tau0 . grad tau1 + tau0 lap tau1,
where tau0's derivatives are analytic, grad tau1 uses central differences (first-order
one-sided on the domain boundary) and lap tau1 the central second difference
(second-order one-sided second difference on the boundary).

Readings where the paper is silent (listed in the design notes):
* at the source node tau0 = 0 and grad tau0 is undefined: grad tau := 0 there and
  lap tau := the 2d-neighbour discrete Laplacian of tau at the source;
* tau1 = tau/tau0 is 0/0 at the source; there it is the mean of tau/tau0 over the
  source's 2d axis neighbours (tau0 = h there).  For tau = kappa(x0) r + O(r^2) this is
  kappa(x0) + O(h^2) (the first-order terms of opposite neighbours cancel), exact for a
  constant medium, and it is a function of tau alone: at fixed tau the operator depends
  on kappa^2 only through the reaction term below, which is what the kappa^2 gradient at
  fixed tau differentiates;
* the reaction: Sec. 1 notes that a travel time solving the eikonal equation removes
  the term -w^2(|grad tau|^2 - kappa^2) from eq. ADR.  Two forms are offered:
  "numerical" keeps it with the numerical grad tau (the discrete system stays a diagonal
  rescaling of the Helmholtz one up to the eikonal residual, and kappa^2 enters the
  operator there), "eikonal" drops it as Sec. 1 does.  Both add the absorbing-layer
  term -i w gamma kappa^2 of Sec. 1:
      numerical: c = w^2 (kappa^2 - |g|^2) - i w gamma kappa^2
      eikonal:   c = -i w gamma kappa^2.
"""
import numpy as np


def first_difference(f, axis, h):
    """d f / d x_axis: central (f[j+1]-f[j-1])/(2h) inside, first-order one-sided at the
    two end nodes (Sec. 2.1)."""
    f = np.moveaxis(np.asarray(f, dtype=np.float64), axis, 0)
    out = np.empty_like(f)
    out[1:-1] = (f[2:] - f[:-2]) / (2.0 * h)
    out[0] = (f[1] - f[0]) / h
    out[-1] = (f[-1] - f[-2]) / h
    return np.moveaxis(out, 0, axis)


def second_difference(f, axis, h):
    """d^2 f / d x_axis^2: central (f[j+1]-2f[j]+f[j-1])/h^2 inside; at the ends the
    second-order one-sided (2f0 - 5f1 + 4f2 - f3)/h^2 and its mirror (Sec. 2.1)."""
    f = np.moveaxis(np.asarray(f, dtype=np.float64), axis, 0)
    if f.shape[0] < 4:
        raise ValueError("one-sided second difference needs >= 4 nodes per axis")
    out = np.empty_like(f)
    out[1:-1] = (f[2:] - 2.0 * f[1:-1] + f[:-2]) / (h * h)
    out[0] = (2.0 * f[0] - 5.0 * f[1] + 4.0 * f[2] - f[3]) / (h * h)
    out[-1] = (2.0 * f[-1] - 5.0 * f[-2] + 4.0 * f[-3] - f[-4]) / (h * h)
    return np.moveaxis(out, 0, axis)


def travel_time_derivatives(tau, h, src=None):
    """Return (g, L): g is a list with one array per NumPy axis (g[a] = d tau / d x_a),
    L = lap tau.

    src None: plain differences of tau itself (no factoring).  Otherwise factored form
    of eq. (travel_time_coeff) with tau0 = |x - x_src|."""
    tau = np.asarray(tau, dtype=np.float64)
    d = tau.ndim
    if src is None:
        g = [first_difference(tau, a, h) for a in range(d)]
        L = sum(second_difference(tau, a, h) for a in range(d))
        return g, L

    src = tuple(int(s) for s in src)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in tau.shape], indexing="ij")
    dx = [(grids[a] - src[a]) * h for a in range(d)]
    r = np.sqrt(sum(x * x for x in dx))
    at_src = r == 0.0
    r_safe = np.where(at_src, 1.0, r)

    tau0 = r
    grad_tau0 = [np.where(at_src, 0.0, x / r_safe) for x in dx]
    lap_tau0 = np.where(at_src, 0.0, (d - 1) / r_safe)

    tau1 = np.where(at_src, 0.0, tau / r_safe)
    nbrs = []
    for a in range(d):
        for o in (-1, 1):
            j = list(src)
            j[a] += o
            nbrs.append(tau1[tuple(j)])
    tau1[src] = np.mean(nbrs)

    grad_tau1 = [first_difference(tau1, a, h) for a in range(d)]
    lap_tau1 = sum(second_difference(tau1, a, h) for a in range(d))

    g = [tau0 * grad_tau1[a] + tau1 * grad_tau0[a] for a in range(d)]
    L = tau1 * lap_tau0 + 2.0 * sum(grad_tau0[a] * grad_tau1[a] for a in range(d)) + tau0 * lap_tau1

    # Source node: grad tau := 0, lap tau := discrete Laplacian of tau there.
    lap_src = 0.0
    for a in range(d):
        e = [0] * d
        e[a] = 1
        plus = tuple(s + o for s, o in zip(src, e))
        minus = tuple(s - o for s, o in zip(src, e))
        lap_src += (tau[plus] - 2.0 * tau[src] + tau[minus]) / (h * h)
    for a in range(d):
        g[a][src] = 0.0
    L[src] = lap_src
    return g, L


def reaction(g, kappa2, gamma, omega, form="numerical"):
    """The reaction coefficient of eq. ADR plus the absorbing term:
    "numerical": c = w^2 (kappa^2 - |g|^2) - i w gamma kappa^2;
    "eikonal":   c = -i w gamma kappa^2 (the eikonal equation removes the w^2 term)."""
    kappa2 = np.asarray(kappa2, dtype=np.float64)
    gam = np.zeros_like(kappa2) if gamma is None else np.asarray(gamma, dtype=np.float64)
    absorb = -1j * omega * gam * kappa2
    if form == "eikonal":
        return absorb + 0.0
    if form != "numerical":
        raise ValueError(form)
    gg = sum(ga * ga for ga in g)
    return omega * omega * (kappa2 - gg) + absorb


def reaction_derivative(gamma, omega, shape, form="numerical"):
    """d c / d kappa^2 at fixed tau, per node: w^2 - i w gamma ("numerical") or
    -i w gamma ("eikonal")."""
    gam = np.zeros(shape) if gamma is None else np.asarray(gamma, dtype=np.float64)
    return (0.0 if form == "eikonal" else omega * omega) - 1j * omega * gam


def adr_coefficients(tau, kappa2, gamma, h, omega, src=None, form="numerical"):
    """All per-node coefficients of the ADR operator: (g list, L, c complex)."""
    g, L = travel_time_derivatives(tau, h, src=src)
    c = reaction(g, kappa2, gamma, omega, form)
    return g, L, c
