"""Pins of the oracle's Krylov cycle (Sec. 3.1, Alg. KrylovCycle; threshold Sec. 4.2.2).

The cycle is data dependent, so it is pinned by properties fixed by its definition:
the W structure of its recursive calls, scale invariance, the minimal-residual property
of each coarse flexible GMRES(2) checked by brute force over the span of its
preconditioned directions, reduction to a two-grid cycle when the coarse preconditioner
is exact, and convergence of the outer solve to the direct solution.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import multigrid, solve
from paper_1712_06091_amd import workloads as W


def _problem(n=33, d=2, seed=7):
    wl = W.random_medium(n, d, seed=seed)
    return solve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src), wl


def _rhs(N, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(N) + 1j * rng.standard_normal(N)


@pytest.mark.parametrize("threshold, expect", [(0.0, [1, 2, 4, 0]), (1.0, [1, 1, 1, 0])])
def test_kcycle_call_structure(threshold, expect):
    """Two coarse Krylov steps per level give the W-cycle's call counts (1, 2, 4 cycles
    on levels 0, 1, 2; the coarsest is solved directly); a threshold of 1 always stops
    after the first step (its residual never exceeds the initial one)."""
    p, _ = _problem()
    hier = p.hierarchy(levels=4)
    hier.kcalls = [0] * 4
    hier.kcycle(_rhs(p.H2up.shape[0]), threshold=threshold)
    assert hier.kcalls == expect


def test_kcycle_two_levels_is_vcycle():
    """With two levels the coarse problem is the coarsest one: no Krylov step, the cycle
    is the two-grid cycle."""
    p, _ = _problem()
    hier = p.hierarchy(levels=2)
    b = _rhs(p.H2up.shape[0], 1)
    np.testing.assert_array_equal(hier.kcycle(b), hier.vcycle(b))


def test_kcycle_scale_invariant():
    """Every step (GMRES relaxation and flexible GMRES from zero, transfers, the exact
    coarsest solve, the threshold test on a ratio) is homogeneous: K(alpha b) = alpha K(b)
    for complex alpha."""
    p, _ = _problem()
    hier = p.hierarchy(levels=4)
    b = _rhs(p.H2up.shape[0], 2)
    alpha = 0.37 - 2.1j
    x1 = hier.kcycle(b)
    x2 = hier.kcycle(alpha * b)
    np.testing.assert_allclose(x2, alpha * x1, rtol=0, atol=1e-11 * np.abs(x1).max() * abs(alpha))


def test_coarse_fgmres_minimizes_residual_over_its_directions():
    """The coarse correction minimizes ||r - A_c e|| over the span of the preconditioned
    directions it generated (recorded here); checked against a dense least-squares fit,
    and the second direction is the cycle applied to the normalized orthogonal
    complement of A_c z_1 against r."""
    p, _ = _problem()
    hier = p.hierarchy(levels=4)
    A1 = hier.A[1]
    r = _rhs(A1.shape[0], 3)
    seen = []
    orig = hier.kcycle

    def recording(b, l=0, threshold=0.1):
        x = orig(b, l, threshold)
        if l == 1:
            seen.append((b.copy(), x.copy()))
        return x

    hier.kcycle = recording
    e = hier.coarse_fgmres(1, r, 0.0)
    hier.kcycle = orig
    assert len(seen) == 2
    (v1, z1), (v2, z2) = seen
    np.testing.assert_allclose(v1, r / np.linalg.norm(r), rtol=0, atol=1e-14)
    w = A1 @ z1
    q = w - np.vdot(v1, w) * v1
    np.testing.assert_allclose(v2, q / np.linalg.norm(q), rtol=0, atol=1e-12)
    M = np.stack([A1 @ z1, A1 @ z2], axis=1)
    c, *_ = np.linalg.lstsq(M, r, rcond=None)
    best = np.linalg.norm(r - M @ c)
    assert abs(np.linalg.norm(r - A1 @ e) - best) <= 1e-10 * np.linalg.norm(r)
    np.testing.assert_allclose(e, np.stack([z1, z2], axis=1) @ c, rtol=0, atol=1e-9 * np.abs(e).max())


def test_kcycle_with_exact_coarse_preconditioner_is_two_grid():
    """If the cycle on level 1 were the exact inverse, the first Krylov step would solve
    the coarse problem exactly (its Hessenberg subdiagonal vanishes), and the Krylov cycle
    would be the two-grid cycle with an exact coarse solve, i.e. the V-cycle of a
    two-level hierarchy on the same fine operator."""
    p, _ = _problem()
    hier = p.hierarchy(levels=4)
    two = p.hierarchy(levels=2)
    lu = spla.splu(hier.A[1].tocsc())
    orig = hier.kcycle

    def exact_on_level1(b, l=0, threshold=0.1):
        if l == 1:
            return lu.solve(b)
        return orig(b, l, threshold)

    hier.kcycle = exact_on_level1
    b = _rhs(p.H2up.shape[0], 4)
    x = hier.kcycle(b)
    hier.kcycle = orig
    ref = two.vcycle(b)
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("d, n", [(2, 65), (3, 17)])
def test_kcycle_solve_matches_direct(d, n):
    """FGMRES(5) preconditioned by the Krylov cycle reaches the direct solution."""
    p, wl = _problem(n, d, seed=5)
    qh = solve.rhs_hat(wl.rhs(), wl.tau, wl.omega)
    a, info = solve.iterative_solve(p, qh, tol=1e-11, maxit=300, cycle="k")
    ref = solve.direct_solve(p.H2up, qh).reshape(p.shape)
    assert info["relres"] <= 1e-11
    assert np.linalg.norm(a - ref) <= 1e-9 * np.linalg.norm(ref)


def test_kcycle_fewer_iterations_than_vcycle():
    """On a heterogeneous 2D medium the Krylov cycle needs fewer outer iterations."""
    p, wl = _problem(129, 2, seed=11)
    qh = solve.rhs_hat(wl.rhs(), wl.tau, wl.omega)
    _, iv = solve.iterative_solve(p, qh, tol=1e-6, maxit=300, cycle="v")
    _, ik = solve.iterative_solve(p, qh, tol=1e-6, maxit=300, cycle="k")
    assert ik["iters"] < iv["iters"]


def test_kcycle_krylov_levels_limit():
    """kmax limits the flexible-GMRES coarse solves to coarse levels 1..kmax: the call
    counts are the W pattern down to level kmax and single calls below it; below kmax the
    cycle is exactly the V-cycle; kmax at or beyond the last relaxed level is the full
    Krylov cycle."""
    p, _ = _problem(n=65)
    hier = p.hierarchy(levels=5)
    b = _rhs(p.H2up.shape[0], 11)
    hier.kcalls = [0] * 5
    hier.kcycle(b, threshold=0.0, kmax=1)
    assert hier.kcalls == [1, 2, 2, 2, 0]
    rc = hier.P[1].T @ (hier.P[0].T @ b)
    np.testing.assert_array_equal(hier.kcycle(rc, l=2, kmax=1), hier.vcycle(rc, l=2))
    np.testing.assert_array_equal(hier.kcycle(b, kmax=3), hier.kcycle(b))
    assert not np.array_equal(hier.kcycle(b, kmax=1), hier.kcycle(b))
