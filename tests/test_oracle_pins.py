"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of them re-types the oracle's formulas: they use
closed forms, exactness of difference formulas on polynomials, an independently built
standard Helmholtz matrix, convergence orders, brute force and library solvers.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.special import hankel2

from oracle import closed_form, coefficients, krylov, multigrid, operators, solve
from paper_1712_06091_amd import workloads as W
from tests.oracle_helpers import boundary_mask, solve_dirichlet


# ----------------------------------------------------------------------------------
# Difference formulas (Sec. 2.1)
# ----------------------------------------------------------------------------------

def test_first_difference_exactness():
    """Central differences are exact for quadratics inside, one-sided ones for lines."""
    h = 0.1
    x = np.arange(9) * h
    q = 2.0 - 3.0 * x + 5.0 * x ** 2
    d = coefficients.first_difference(q, 0, h)
    np.testing.assert_allclose(d[1:-1], (-3.0 + 10.0 * x)[1:-1], rtol=0, atol=1e-12)
    lin = 1.5 - 4.0 * x
    np.testing.assert_allclose(coefficients.first_difference(lin, 0, h), -4.0, atol=1e-12)


def test_second_difference_exactness():
    """Central and one-sided second differences are exact for cubics."""
    h = 0.05
    x = np.arange(11) * h
    cub = 1.0 + 2.0 * x - 3.0 * x ** 2 + 4.0 * x ** 3
    exact = -6.0 + 24.0 * x
    np.testing.assert_allclose(coefficients.second_difference(cub, 0, h), exact, atol=1e-9)


# ----------------------------------------------------------------------------------
# Coefficients (eq. travel_time_coeff)
# ----------------------------------------------------------------------------------

@pytest.mark.parametrize("d", [2, 3])
def test_coefficients_constant_medium_exact(d):
    """kappa constant, tau = kappa r  =>  tau1 == kappa, so g = kappa (x-x0)/r and
    lap tau = kappa (d-1)/r exactly; c = -i w gamma kappa^2; at the source g = 0 and
    lap tau = discrete Laplacian of kappa r = 2 d kappa / h."""
    n = 17 if d == 3 else 33
    shape = (n,) * d
    h = 1.0 / (n - 1)
    kap = 1.3
    src = tuple([n // 2 - 1] + [n // 2] * (d - 1))
    r = W.distance(shape, h, src)
    tau = kap * r
    gam = W.absorbing_layer(shape, h, 40.0, 5 * h)
    g, L, c = coefficients.adr_coefficients(tau, np.full(shape, kap ** 2), gam, h, 40.0, src=src)
    xs = W.node_coordinates(shape, h)
    rs = np.where(r == 0, 1.0, r)
    for a in range(d):
        expect = np.where(r == 0, 0.0, kap * (xs[a] - src[a] * h) / rs)
        np.testing.assert_allclose(g[a], expect, rtol=0, atol=1e-11)
    expectL = np.where(r == 0, 2 * d * kap / h, kap * (d - 1) / rs)
    np.testing.assert_allclose(L, expectL, rtol=1e-12, atol=1e-9)
    # |g|^2 = kappa^2 except at the source, where g := 0 leaves w^2 kappa^2.
    expect_c = -1j * 40.0 * gam * kap ** 2 + np.where(r == 0, 40.0 ** 2 * kap ** 2, 0.0)
    np.testing.assert_allclose(c, expect_c, rtol=0, atol=1e-8)


def _tau_linear(points, src_pos, v0, G):
    depth = points[0]
    v = v0 + G * depth
    vs = v0 + G * src_pos[0]
    r2 = sum((p - s) ** 2 for p, s in zip(points, src_pos))
    return np.arccosh(1.0 + G * G * r2 / (2.0 * v * vs)) / G


def test_coefficients_linear_gradient_second_order():
    """v = 1.5 + 0.8 depth (closed-form tau): the eikonal residual | |g|^2 - kappa^2 |
    and the error of L against lap tau (4th-order differences of the closed form with a
    tiny step) fall at second order away from the source and the faces."""
    errs_e, errs_l = [], []
    for n in (33, 65):
        wl = W.linear_gradient(n, ndim=2, absorb=False)
        g, L = coefficients.travel_time_derivatives(wl.tau, wl.h, src=wl.src)
        xs = W.node_coordinates(wl.shape, wl.h)
        r = W.distance(wl.shape, wl.h, wl.src)
        mask = (r >= 0.2) & ~boundary_mask(wl.shape)
        eik = np.abs(g[0] ** 2 + g[1] ** 2 - wl.kappa2)[mask]
        src_pos = [s * wl.h for s in wl.src]
        e = 1e-3
        lap = 0.0
        for a in range(2):
            def shifted(k):
                p = [x.copy() for x in xs]
                p[a] = p[a] + k * e
                return _tau_linear(p, src_pos, 1.5, 0.8)
            lap = lap + (-shifted(2) + 16 * shifted(1) - 30 * shifted(0) + 16 * shifted(-1) - shifted(-2)) / (12 * e * e)
        errs_e.append(eik.max())
        errs_l.append(np.abs(L - lap)[mask].max())
    assert np.log2(errs_e[0] / errs_e[1]) > 1.8
    assert np.log2(errs_l[0] / errs_l[1]) > 1.7


# ----------------------------------------------------------------------------------
# Operators (Sec. 2.2-2.3, eq. BCADR, eq. precADRup)
# ----------------------------------------------------------------------------------

@pytest.mark.parametrize("d,beta", [(2, 0.0), (2, 0.25), (3, 1.0), (3, 0.25)])
def test_tau_zero_gives_helmholtz(d, beta):
    """tau = 0 turns the ADR system back into the Helmholtz system exactly (Sec. 1):
    A_beta must equal the independently built Kronecker-sum H entry by entry."""
    n = 9 if d == 3 else 17
    shape = (n,) * d
    h = 1.0 / (n - 1)
    rng = np.random.default_rng(1)
    kappa2 = 0.5 + rng.random(shape)
    gam = W.absorbing_layer(shape, h, 30.0, 3 * h)
    g, L, c = coefficients.adr_coefficients(np.zeros(shape), kappa2, gam, h, 30.0, src=None)
    A = operators.assemble_adr(g, L, c, h, 30.0, beta, src=None)
    H = operators.assemble_helmholtz(kappa2, gam, h, 30.0)
    assert abs(A - H).max() == 0.0


def _quadratic(shape, h, seed):
    """Random complex quadratic a(x) with its gradient and Laplacian on the nodes."""
    rng = np.random.default_rng(seed)
    d = len(shape)
    xs = W.node_coordinates(shape, h)
    lin = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    Q = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    Q = Q + Q.T
    a = 0.3 + 0.2j + sum(lin[i] * xs[i] for i in range(d))
    a = a + 0.5 * sum(Q[i, j] * xs[i] * xs[j] for i in range(d) for j in range(d))
    grad = [lin[i] + sum(Q[i, j] * xs[j] for j in range(d)) for i in range(d)]
    second = [Q[i, i] * np.ones(shape) for i in range(d)]
    return a, grad, second


@pytest.mark.parametrize("d,beta", [(2, 0.0), (2, 0.25), (2, 1.0), (3, 0.25)])
def test_operator_on_quadratics(d, beta):
    """On quadratics the Laplacian, the second-order upwind and central differences are
    exact, the first-order upwind one is a' -+ (h/2) a'' and the isotropic average is
    a + h^2/(2d) lap a.  Random coefficient fields with both signs of g exercise the
    upwind direction; rows next to the source use central differences (Sec. 2.2)."""
    n = 11 if d == 3 else 21
    shape = (n,) * d
    h = 1.0 / (n - 1)
    omega = 7.0
    rng = np.random.default_rng(2)
    g = [rng.standard_normal(shape) for _ in range(d)]
    L = rng.standard_normal(shape)
    c = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    src = (n // 2,) * d
    A = operators.assemble_adr(g, L, c, h, omega, beta, src=src)
    a, grad, second = _quadratic(shape, h, 3)
    got = (A @ a.ravel()).reshape(shape)
    idx = np.meshgrid(*[np.arange(k) for k in shape], indexing="ij")
    cheb = np.max(np.stack([np.abs(idx[k] - src[k]) for k in range(d)]), axis=0)
    inner = np.ones(shape, dtype=bool)
    for k in range(d):
        inner &= (idx[k] >= 2) & (idx[k] <= n - 3)
    lap = sum(second)
    adv = 0.0
    for k in range(d):
        sign = np.where(g[k] >= 0, 1.0, -1.0)            # backward for g >= 0
        dk = np.where(cheb <= 1, grad[k], grad[k] - beta * sign * 0.5 * h * second[k])
        adv = adv + g[k] * dk
    expect = lap - 2j * omega * adv - 1j * omega * L * (a + h * h / (2 * d) * lap) + c * a
    np.testing.assert_allclose(got[inner], expect[inner], rtol=1e-11, atol=1e-8)


@pytest.mark.parametrize("d,beta", [(2, 0.0), (2, 0.25), (3, 0.25), (3, 1.0)])
def test_operator_rows_one_node_from_faces(d, beta):
    """Rows one node inside a face whose upwind stencil would need the node beyond the
    face (g_k > 0 at i_k = 1, g_k < 0 at i_k = n-2): both upwind orders fall back to the
    first-order upwind difference, whose value on a quadratic is a' -+ (h/2) a''
    whatever beta.  Every row off the faces is checked, on every axis, with random
    coefficient signs; rows that do not fall back follow the interior rules."""
    n = 9 if d == 3 else 15
    shape = (n,) * d
    h = 1.0 / (n - 1)
    omega = 6.0
    rng = np.random.default_rng(12)
    g = [rng.standard_normal(shape) for _ in range(d)]
    L = rng.standard_normal(shape)
    c = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    src = (n // 2,) * d
    A = operators.assemble_adr(g, L, c, h, omega, beta, src=src)
    a, grad, second = _quadratic(shape, h, 13)
    got = (A @ a.ravel()).reshape(shape)
    idx = np.meshgrid(*[np.arange(k) for k in shape], indexing="ij")
    cheb = np.max(np.stack([np.abs(idx[k] - src[k]) for k in range(d)]), axis=0)
    off_faces = np.ones(shape, dtype=bool)
    for k in range(d):
        off_faces &= (idx[k] >= 1) & (idx[k] <= n - 2)
    lap = sum(second)
    adv = 0.0
    short = np.zeros(shape, dtype=bool)
    for k in range(d):
        back = g[k] >= 0
        one_short_b = back & (idx[k] == 1)
        one_short_f = ~back & (idx[k] == n - 2)
        short |= (one_short_b | one_short_f) & (cheb > 1)
        sign = np.where(back, 1.0, -1.0)
        first_order = grad[k] - sign * 0.5 * h * second[k]
        blended = grad[k] - beta * sign * 0.5 * h * second[k]
        dk = np.where(one_short_b | one_short_f, first_order, blended)
        dk = np.where(cheb <= 1, grad[k], dk)
        adv = adv + g[k] * dk
    expect = lap - 2j * omega * adv - 1j * omega * L * (a + h * h / (2 * d) * lap) + c * a
    assert short[off_faces].sum() > 10
    np.testing.assert_allclose(got[off_faces], expect[off_faces], rtol=1e-11, atol=1e-8)


@pytest.mark.parametrize("g0", [0.7, -0.7])
def test_operator_face_rows(g0):
    """Face rows: a(x) = 1 + i w g0 s + c2 s^2 (s = distance into the domain along x)
    satisfies n.grad a - i w (n.grad tau) a = 0 (eq. BCADR) with g_x = +-g0 on the face,
    so the ghost-node Laplacian row equals a'' exactly; the upwind term uses a one-sided
    stencil exact for quadratics and the mass term uses a itself."""
    n = 13
    shape = (n, n)
    h = 1.0 / (n - 1)
    omega, c2 = 5.0, 0.8 - 0.3j
    rng = np.random.default_rng(4)
    L = rng.standard_normal(shape)
    c = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    Y, X = W.node_coordinates(shape, h)
    for side in (0, 1):
        s = X if side == 0 else 1.0 - X             # distance from the face
        gx = np.full(shape, g0 if side == 0 else -g0)   # BC: d a/dn = i w (n.g) a
        gy = 0.3 * rng.standard_normal(shape)
        a = 1.0 + 1j * omega * g0 * s + c2 * s ** 2
        A = operators.assemble_adr([gy, gx], L, c, h, omega, 0.25, src=None)  # beta = 0.25
        got = (A @ a.ravel()).reshape(shape)
        col = 0 if side == 0 else n - 1
        rows = slice(1, n - 1)
        dadx = (1j * omega * g0) * (1.0 if side == 0 else -1.0)   # a'(face) along +x
        # Face rows always use the inward one-sided pair: second order exact, first
        # order a' +- (h/2) a'' (forward on the low face, backward on the high face).
        beta = 0.25
        dbeta = dadx + beta * 0.5 * h * 2 * c2 * (1.0 if side == 0 else -1.0)
        expect = 2 * c2 - 2j * omega * gx[rows, col] * dbeta - 1j * omega * L[rows, col] + c[rows, col]
        np.testing.assert_allclose(got[rows, col], expect, rtol=1e-12, atol=1e-9)


def _manufactured_error(n, beta, omega=20.0, gam=2.0, x0=(-0.3, -0.2), form="numerical"):
    shape = (n, n)
    h = 1.0 / (n - 1)
    Y, X = W.node_coordinates(shape, h)
    dx, dy = X - x0[0], Y - x0[1]
    r = np.sqrt(dx * dx + dy * dy)
    s1, s2 = np.sin(np.pi * X), np.sin(2 * np.pi * Y)
    c1, c2 = np.cos(np.pi * X), np.cos(2 * np.pi * Y)
    p = 1 + 0.5j * X
    a = s1 * s2 * p
    ax = np.pi * c1 * s2 * p + 0.5j * s1 * s2
    ay = 2 * np.pi * s1 * c2 * p
    lap = -np.pi ** 2 * s1 * s2 * p + 1j * np.pi * c1 * s2 - 4 * np.pi ** 2 * s1 * s2 * p
    # eq. ADR with tau = |x - x0| (|grad tau| = kappa = 1, lap tau = 1/r) and absorption.
    f = lap - 2j * omega * (dx / r * ax + dy / r * ay) - 1j * omega / r * a - 1j * omega * gam * a
    g, L, c = coefficients.adr_coefficients(r, np.ones(shape), np.full(shape, gam), h, omega, src=None, form=form)
    A = operators.assemble_adr(g, L, c, h, omega, beta, src=None)
    ah = solve_dirichlet(A, shape, f, a)
    return np.linalg.norm(ah - a) / np.linalg.norm(a)


@pytest.mark.parametrize("form", ["numerical", "eikonal"])
def test_manufactured_solution_orders(form):
    """Smooth manufactured amplitude, smooth tau solving the eikonal equation (source
    outside the domain, kappa = 1), so eq. ADR has no w^2 reaction term: H_2up converges at
    second order (Sec. 2.2 claims a second-order scheme), H_1up at first, with the
    reaction kept as the numerical eikonal residual or dropped (Sec. 1)."""
    e2 = [_manufactured_error(n, 0.0, form=form) for n in (65, 129, 257)]
    e1 = [_manufactured_error(n, 1.0, form=form) for n in (65, 129)]
    o2 = np.log2(e2[1] / e2[2])
    assert np.log2(e2[0] / e2[1]) > 1.7 and o2 > 1.8
    assert 0.75 < np.log2(e1[0] / e1[1]) < 1.2


def _point_source_errors(n, omega=20.0, gam=2.0):
    shape = (n, n)
    h = 1.0 / (n - 1)
    src = (n // 2, n // 2)
    r = W.distance(shape, h, src)
    rs = np.where(r == 0, 1.0, r)
    k = np.sqrt(omega ** 2 - 1j * omega * gam + 0j)
    k = -k if k.imag > 0 else k                      # decaying exp(-i k r)
    u_exact = 0.25j * hankel2(0, k * rs)
    a_exact = u_exact * np.exp(1j * omega * rs)
    G = np.full(shape, gam)
    g, L, c = coefficients.adr_coefficients(r, np.ones(shape), G, h, omega, src=src)
    A = operators.assemble_adr(g, L, c, h, omega, 0.0, src=src)
    q = solve.point_source_rhs(shape, src, h)
    a = solve_dirichlet(A, shape, solve.rhs_hat(q, r, omega), a_exact)
    H = operators.assemble_helmholtz(np.ones(shape), G, h, omega)
    u = solve_dirichlet(H, shape, q, u_exact)
    m = r >= 0.1
    rel = lambda x, y: np.linalg.norm((x - y)[m]) / np.linalg.norm(y[m])
    return rel(a, a_exact), rel(u, u_exact)


def test_point_source_closed_form():
    """2D constant medium, point source (Sec. 1 closed form with absorption, Dirichlet
    data on the faces): the standard scheme converges at second order (pins the closed
    form's sign and H); the ADR amplitude converges too, at first order -- the
    near-source terms (lap tau ~ 1/r) cap it, a reading recorded in the design notes."""
    e = [_point_source_errors(n) for n in (65, 129, 257)]
    std = [x[1] for x in e]
    adr = [x[0] for x in e]
    assert np.log2(std[0] / std[1]) > 1.9 and np.log2(std[1] / std[2]) > 1.9
    assert adr[2] < adr[1] < adr[0]
    assert np.log2(adr[0] / adr[2]) / 2 > 0.9
    assert adr[2] < 0.05


def test_closed_form_3d_satisfies_pde():
    """-exp(-i w r)/(4 pi r) satisfies Delta u + w^2 u = 0 away from the source (checked
    with a 4th-order difference) and carries unit flux into the source (+delta)."""
    omega = 9.0
    x = np.array([0.31, -0.22, 0.17])
    e = 1e-3
    f = lambda p: closed_form.wavefield_3d(np.linalg.norm(p), omega)
    lap = 0.0
    for a in range(3):
        ea = np.zeros(3)
        ea[a] = e
        lap += (-f(x + 2 * ea) + 16 * f(x + ea) - 30 * f(x) + 16 * f(x - ea) - f(x - 2 * ea)) / (12 * e * e)
    assert abs(lap + omega ** 2 * f(x)) < 1e-6 * abs(omega ** 2 * f(x))
    # Flux through a small sphere: 4 pi r^2 du/dr -> 1 as r -> 0 (so Delta u = +delta).
    r = 1e-6
    dudr = (closed_form.wavefield_3d(r * (1 + 1e-4), omega) - closed_form.wavefield_3d(r * (1 - 1e-4), omega)) / (2e-4 * r)
    assert abs(4 * np.pi * r * r * dudr - 1.0) < 1e-4


def test_closed_form_2d_matches_library():
    """The 2D amplitude is (i/4) H0^(2)(w r) exp(i w r)."""
    r = np.linspace(0.05, 1.0, 7)
    np.testing.assert_allclose(closed_form.amplitude_2d(r, 12.0),
                               0.25j * hankel2(0, 12.0 * r) * np.exp(12j * r), rtol=1e-14)


@pytest.mark.slow
def test_adr_beats_standard_at_10ppw():
    """Sec. 4.1: smooth medium, no reflections: at 10 points per wavelength the ADR
    wavefield u = a exp(-i w tau) is closer to a 4x-finer standard solution than the
    standard scheme on the same grid (thick absorbing layer, interior region)."""
    n, ff, thick = 257, 4, 0.25
    wl = W.linear_gradient(n, ndim=2, src_frac=(0.5, 0.3), absorb=False)
    wf = W.linear_gradient((n - 1) * ff + 1, ndim=2, src_frac=(0.5, 0.3), absorb=False)
    om = wl.omega
    gam = W.absorbing_layer(wl.shape, wl.h, om, thick)
    gamf = W.absorbing_layer(wf.shape, wf.h, om, thick)
    p = solve.Problem(wl.kappa2, wl.tau, gam, wl.h, om, wl.src)
    a = solve.direct_solve(p.H2up, solve.rhs_hat(wl.rhs(), wl.tau, om)).reshape(wl.shape)
    u_adr = solve.wavefield(a, wl.tau, om)
    u_std = solve.direct_solve(operators.assemble_helmholtz(wl.kappa2, gam, wl.h, om), wl.rhs()).reshape(wl.shape)
    u_ref = solve.direct_solve(operators.assemble_helmholtz(wf.kappa2, gamf, wf.h, om),
                               wf.rhs()).reshape(wf.shape)[::ff, ::ff]
    r = W.distance(wl.shape, wl.h, wl.src)
    Y, X = W.node_coordinates(wl.shape, wl.h)
    m = (r >= 0.1) & (X > thick) & (X < 1 - thick) & (Y > thick) & (Y < 1 - thick)
    err = lambda u: np.linalg.norm((u - u_ref)[m]) / np.linalg.norm(u_ref[m])
    assert err(u_adr) < 0.85 * err(u_std)


def test_sign_convention_conjugates():
    """Flipping the sign of w (the other Rytov convention) conjugates the system, so the
    amplitude becomes conj(a) for real kappa^2, gamma and q."""
    wl = W.constant_medium(17, ndim=2)
    p1 = solve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    g, L, c = coefficients.adr_coefficients(wl.tau, wl.kappa2, wl.gamma, wl.h, -wl.omega, src=wl.src)
    A2 = operators.assemble_adr(g, L, c, wl.h, -wl.omega, 0.0, src=wl.src)
    a1 = solve.direct_solve(p1.H2up, solve.rhs_hat(wl.rhs(), wl.tau, wl.omega))
    a2 = solve.direct_solve(A2, solve.rhs_hat(wl.rhs(), wl.tau, -wl.omega))
    np.testing.assert_allclose(a2, np.conj(a1), rtol=1e-12, atol=1e-12 * np.abs(a1).max())


# ----------------------------------------------------------------------------------
# Multigrid and Krylov (Sec. 3)
# ----------------------------------------------------------------------------------

def test_prolongation_exact_on_multilinear():
    shape = (9, 5, 7)
    P = multigrid.prolongation(shape)
    cs = multigrid.coarse_shape(shape)
    xc = W.node_coordinates(cs, 2.0)
    xf = W.node_coordinates(shape, 1.0)
    f = lambda x: 1.0 + 2 * x[0] - x[1] + 0.5 * x[2] + 0.3 * x[0] * x[1] * x[2] - x[1] * x[2]
    np.testing.assert_allclose(P @ f(xc).ravel(), f(xf).ravel(), rtol=1e-13, atol=1e-12)


def test_galerkin_laplacian_closed_form():
    """1D: P^T (h^-2 [1 -2 1]) P = (2h)^-2 * 2 [1 -2 1] on interior coarse rows
    (P^T is twice full weighting)."""
    n = 17
    h = 0.1
    A = sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1]) / h ** 2
    P = multigrid.prolongation_1d(n)
    Ac = (P.T @ A @ P).toarray()
    H2 = (2 * h) ** 2
    for I in range(1, Ac.shape[0] - 1):
        np.testing.assert_allclose(Ac[I, I - 1:I + 2], 2 * np.array([1, -2, 1]) / H2, rtol=1e-13)


def _small_problem(n=33):
    wl = W.linear_gradient(n, ndim=2)
    return wl, solve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)


def test_galerkin_support_81_and_21():
    """Galerkin coarse operators keep the support: 21 points in 2D, 81 in 3D (offsets
    with at most one coordinate of magnitude 2)."""
    wl, p = _small_problem(33)
    hier = p.hierarchy(3)
    for l in (1, 2):
        A = hier.A[l].tocoo()
        ns = hier.shapes[l]
        ri = np.array(np.unravel_index(A.row, ns))
        ci = np.array(np.unravel_index(A.col, ns))
        offs = {tuple(o) for o in (ci - ri).T}
        assert len(offs) <= 21
        assert all(sum(abs(x) == 2 for x in o) <= 1 and max(abs(x) for x in o) <= 2 for o in offs)
    wl3 = W.linear_gradient(17, ndim=3)
    p3 = solve.Problem(wl3.kappa2, wl3.tau, wl3.gamma, wl3.h, wl3.omega, wl3.src)
    h3 = p3.hierarchy(2)
    A = h3.A[1].tocoo()
    ns = h3.shapes[1]
    ri = np.array(np.unravel_index(A.row, ns))
    ci = np.array(np.unravel_index(A.col, ns))
    offs = {tuple(o) for o in (ci - ri).T}
    assert len(offs) == 81


def test_gmres_relaxation_is_residual_minimizer():
    """GMRES relaxation returns the minimizer of ||b - A(x + D^-1 K y)|| over the Krylov
    space K of A D^-1 and r; brute force with explicit Krylov powers agrees."""
    wl, p = _small_problem(17)
    hier = p.hierarchy(2)
    A, dinv = hier.A[1], hier.dinv[1]
    rng = np.random.default_rng(5)
    b = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    x0 = rng.standard_normal(A.shape[0]) * 0.1 + 0j
    x1 = hier.gmres_relax(1, x0, b, 3)
    r = b - A @ x0
    K = [r]
    for _ in range(2):
        K.append(A @ (dinv * K[-1]))
    K = np.array(K).T
    M = A @ (dinv[:, None] * K)
    y = np.linalg.lstsq(M, r, rcond=None)[0]
    x_bf = x0 + dinv * (K @ y)
    np.testing.assert_allclose(x1, x_bf, rtol=1e-8, atol=1e-10 * np.abs(x_bf).max())
    assert np.linalg.norm(b - A @ x1) < np.linalg.norm(b - A @ x0)


def _dense_prolongation(shape):
    """Nodal (bi/tri)linear interpolation as a dense matrix, built from its definition:
    the fine node x takes the coarse values at the corners of its coarse cell, each
    weighted by the product over axes of (1 - |x_k - 2 X_k| / 2)."""
    cs = tuple((n - 1) // 2 + 1 for n in shape)
    fine = np.array(np.unravel_index(np.arange(int(np.prod(shape))), shape)).T
    coarse = np.array(np.unravel_index(np.arange(int(np.prod(cs))), cs)).T
    P = np.ones((len(fine), len(coarse)))
    for k in range(len(shape)):
        dist = np.abs(fine[:, k][:, None] - 2 * coarse[:, k][None, :]) / 2.0
        P *= np.clip(1.0 - dist, 0.0, None)
    return P, cs


@pytest.mark.parametrize("levels", [2, 3])
def test_vcycle_is_the_two_grid_recursion(levels):
    """With damped Jacobi on every level the V-cycle from a zero guess is a linear map
    B, and Alg. TwoCycle fixes it: the error propagation of the cycle on level l is
    E_l = S_l^nu (I - P B_{l+1} P^T A_l) S_l^nu with S_l = I - w D_l^-1 A_l, the coarse
    operator P^T A_l P, B_L = A_L^-1 on the coarsest level and B_l = (I - E_l) A_l^-1.
    Built here with dense matrices and an independently written interpolation; the
    oracle's V-cycle must reproduce B_0 b.  Dropping a relaxation, the coarse
    correction, or transposing P changes the result."""
    wl = W.linear_gradient(17, ndim=2)
    p = solve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    nu = [2, 3, 4][:levels]
    w = 0.8
    hier = p.hierarchy(levels, nu=nu, jacobi_weight=w, smoothers=["jacobi"] * levels)
    A = [p.Abeta.toarray()]
    Ps = []
    shape = wl.shape
    for _ in range(levels - 1):
        P, shape = _dense_prolongation(shape)
        Ps.append(P)
        A.append(P.T @ A[-1] @ P)
    B = np.linalg.inv(A[-1])
    for l in range(levels - 2, -1, -1):
        I = np.eye(A[l].shape[0])
        S = I - w * np.diag(1.0 / np.diag(A[l])) @ A[l]
        Sn = np.linalg.matrix_power(S, nu[l])
        E = Sn @ (I - Ps[l] @ B @ Ps[l].T @ A[l]) @ Sn
        B = (I - E) @ np.linalg.inv(A[l])
    rng = np.random.default_rng(21)
    b = rng.standard_normal(A[0].shape[0]) + 1j * rng.standard_normal(A[0].shape[0])
    x = hier.vcycle(b)
    ref = B @ b
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_jacobi_fixed_point():
    wl, p = _small_problem(17)
    hier = p.hierarchy(2)
    x = solve.direct_solve(hier.A[0], np.ones(hier.A[0].shape[0]))
    x2 = hier.jacobi(0, x, np.ones(hier.A[0].shape[0]), 3)
    np.testing.assert_allclose(x2, x, rtol=1e-10, atol=1e-12 * np.abs(x).max())


def test_fgmres_exact_in_k_steps():
    """A diagonal matrix with 4 distinct eigenvalues: GMRES converges in <= 4 steps."""
    ev = np.array([1.0, 2.0 + 1j, -3.0, 0.5j])
    d = np.repeat(ev, 25)
    b = np.random.default_rng(6).standard_normal(100) + 0j
    x, info = krylov.fgmres(lambda v: d * v, b, restart=5, tol=1e-12, maxit=10)
    assert info["iters"] <= 4
    np.testing.assert_allclose(x, b / d, rtol=1e-10)


@pytest.mark.parametrize("d,n", [(2, 65), (3, 17)])
def test_direct_and_iterative_solves_agree(d, n):
    """Check B: dense LU / sparse LU of H_2up and the V-cycle-preconditioned FGMRES
    (driven to 1e-12) give the same amplitude."""
    wl = W.linear_gradient(n, ndim=d)
    p = solve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    qh = solve.rhs_hat(wl.rhs(), wl.tau, wl.omega)
    a_dir = solve.direct_solve(p.H2up, qh)
    a_it, info = solve.iterative_solve(p, qh, tol=1e-12)
    assert info["relres"] <= 1e-12
    assert np.linalg.norm(a_it.ravel() - a_dir) / np.linalg.norm(a_dir) < 1e-9
    if p.H2up.shape[0] <= 5000:
        a_sp = sp.linalg.splu(p.H2up.tocsc()).solve(qh.ravel())
        assert np.linalg.norm(a_sp - a_dir) / np.linalg.norm(a_dir) < 1e-11


def test_vcycle_preconditioner_converges_2d_129():
    """The 2D 129^2 kappa = 1 workload: FGMRES(5) + V-cycle reaches 1e-6 in < 60 steps."""
    wl = W.config_2d_129()
    p = solve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    a, info = solve.iterative_solve(p, solve.rhs_hat(wl.rhs(), wl.tau, wl.omega), tol=1e-6)
    assert info["relres"] <= 1e-6 and info["iters"] < 60


# ----------------------------------------------------------------------------------
# Adjoint (gradient of a receiver misfit w.r.t. kappa^2 at fixed tau)
# ----------------------------------------------------------------------------------

@pytest.mark.parametrize("form", ["numerical", "eikonal"])
def test_adjoint_gradient_finite_differences(form):
    """The adjoint gradient equals central finite differences of the whole forward map
    kappa^2 -> J at fixed tau (coefficients rebuilt from the perturbed kappa^2), in a
    direction that is nonzero everywhere, the source node included: at fixed tau the
    operator may depend on kappa^2 only through its reaction term (with the eikonal form,
    only through the absorbing term)."""
    wl = W.linear_gradient(17, ndim=2)
    rec = (np.full(8, 1), np.arange(1, 17, 2))
    rng = np.random.default_rng(7)
    d_obs = rng.standard_normal(len(rec[0])) * 0.01 + 0j

    def solve_for(k2):
        p = solve.Problem(k2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src, reaction=form)
        a = solve.direct_solve(p.H2up, solve.rhs_hat(wl.rhs(), wl.tau, wl.omega)).reshape(wl.shape)
        return p, a

    p, a = solve_for(wl.kappa2)
    J, grad, _ = solve.adjoint_gradient(p, a, rec, d_obs)
    dk = rng.standard_normal(wl.shape)
    assert abs(dk[wl.src]) > 0.1
    for direction in (dk, np.where(np.arange(dk.size).reshape(wl.shape) == np.ravel_multi_index(wl.src, wl.shape),
                                   1.0, 0.0)):
        eps = 1e-6
        vals = []
        for s in (+1, -1):
            _, aa = solve_for(wl.kappa2 + s * eps * direction)
            u = solve.wavefield(aa, wl.tau, wl.omega)
            vals.append(0.5 * np.sum(np.abs(u[rec] - d_obs) ** 2))
        fd = (vals[0] - vals[1]) / (2 * eps)
        an = float(np.sum(grad * direction))
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-14 * abs(J)
