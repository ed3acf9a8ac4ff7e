"""GPU parity of the Krylov cycle (Alg. KrylovCycle): one cycle through the C ABI
against the oracle's cycle, and whole solves against the direct solution.

Every case prints its name and sizes before touching the GPU.
"""
import numpy as np
import pytest

from oracle import solve as osolve
from paper_1712_06091_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _ctx(wl, prec="fp64", **opts):
    from paper_1712_06091_amd import adr
    o = adr.default_options(prec=prec, cycle="k", **opts)
    gamma = _t(wl.gamma, torch.float64) if wl.gamma is not None else None
    return adr.Context(_t(wl.kappa2, torch.float64), _t(wl.tau, torch.float64), gamma, wl.h, wl.omega, wl.src,
                       options=o)


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _noncubic():
    shape = (17, 25, 33)
    h = 1.0 / 32
    src = (5, 12, 16)
    xs = W.node_coordinates(shape, h)
    v = 1.5 + 0.8 * xs[0]
    tau = W.linear_velocity_traveltime(shape, h, src, 1.5, 0.8)
    omega = W.omega_for_ppw(1.5, h)
    return W.Workload("noncubic", shape, h, omega, src, 1.0 / v ** 2, tau,
                      W.absorbing_layer(shape, h, omega, 4 * h))


# (workload, levels): Krylov steps on levels 1..levels-2
CASES = {
    "2d_129_rand_5lv": (lambda: W.random_medium(129, 2, seed=21), 5),
    "2d_65_const_4lv": (lambda: W.constant_medium(65, 2), 4),
    "3d_33_lin_3lv": (lambda: W.linear_gradient(33, 3), 3),
    "3d_noncubic_3lv": (_noncubic, 3),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("threshold", [0.1, 1.0])
def test_kcycle_fp64(name, threshold):
    """One Krylov cycle equals the oracle's up to rounding; threshold 1 makes every
    coarse GMRES keep only its first step."""
    make, levels = CASES[name]
    wl = make()
    print(f"[kcycle-fp64] {name} shape={wl.shape} threshold={threshold}", flush=True)
    ctx = _ctx(wl, prec="fp64", levels=levels, kcycle_threshold=threshold)
    assert ctx.num_levels == levels
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(levels)
    r = W.random_vector(wl.shape, 31)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    ref = hier.kcycle(r.ravel(), threshold=threshold).reshape(wl.shape)
    assert _rel(z, ref) <= 1e-10


@pytest.mark.parametrize("name", ["2d_129_rand_5lv", "3d_33_lin_3lv"])
def test_kcycle_mixed_close(name):
    """The complex-FP32 Krylov cycle stays within FP32 rounding of the FP64 one."""
    make, levels = CASES[name]
    wl = make()
    print(f"[kcycle-mixed] {name} shape={wl.shape}", flush=True)
    ctx = _ctx(wl, prec="mixed", levels=levels)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(levels)
    r = W.random_vector(wl.shape, 32)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    ref = hier.kcycle(r.ravel()).reshape(wl.shape)
    assert _rel(z, ref) <= 1e-4


def test_kcycle_homogeneous():
    """Scaling the input by a complex factor scales the output (FP64)."""
    make, levels = CASES["2d_129_rand_5lv"]
    wl = make()
    print(f"[kcycle-scale] shape={wl.shape}", flush=True)
    ctx = _ctx(wl, prec="fp64", levels=levels)
    r = W.random_vector(wl.shape, 33)
    alpha = 0.37 - 2.1j
    z1 = ctx.vcycle(_t(r)).cpu().numpy()
    z2 = ctx.vcycle(_t(alpha * r)).cpu().numpy()
    assert _rel(z2, alpha * z1) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_kcycle_solve_matches_direct(prec):
    """FGMRES(5) with the Krylov cycle reaches the direct solution; in FP64 its iteration
    count at tol 1e-6 is the oracle's."""
    make, levels = CASES["2d_129_rand_5lv"]
    wl = make()
    print(f"[kcycle-solve] shape={wl.shape} prec={prec}", flush=True)
    ctx = _ctx(wl, prec=prec, levels=levels)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    qh = osolve.rhs_hat(wl.rhs(), wl.tau, wl.omega)
    ref = osolve.direct_solve(p.H2up, qh).reshape(wl.shape)
    a, st = ctx.solve(_t(wl.rhs()), tol=1e-10, maxit=300)
    a = a.cpu().numpy()
    assert st["relres"] <= 1e-10
    assert np.linalg.norm(p.H2up @ a.ravel() - qh.ravel()) / np.linalg.norm(qh) <= 2e-10
    assert _rel(a, ref) <= 1e-6
    if prec == "fp64":
        _, st6 = ctx.solve(_t(wl.rhs()), tol=1e-6, maxit=300)
        _, info = osolve.iterative_solve(p, qh, levels=levels, tol=1e-6, maxit=300, cycle="k")
        assert abs(st6["outer_iters"] - info["iters"]) <= 1


def test_kcycle_graph_replays_match_eager():
    """The captured cycle replays bitwise like eager launches, several times in a row."""
    make, levels = CASES["2d_129_rand_5lv"]
    wl = make()
    print(f"[kcycle-graph] shape={wl.shape}", flush=True)
    eager = _ctx(wl, prec="mixed", levels=levels, use_graph=0)
    graph = _ctx(wl, prec="mixed", levels=levels, use_graph=1)
    a0, s0 = eager.solve(_t(wl.rhs()), tol=1e-8, maxit=300)
    for _ in range(3):
        a1, s1 = graph.solve(_t(wl.rhs()), tol=1e-8, maxit=300)
        torch.cuda.synchronize()
        assert s1["outer_iters"] == s0["outer_iters"]
        assert torch.equal(a1, a0)


def test_kcycle_adjoint_solve():
    """The adjoint solve with the Krylov cycle on the conjugate-transposed hierarchy
    reaches the direct solution of H_2up^H lam = g exp(i w tau)."""
    wl = W.random_medium(65, 2, seed=22)
    print(f"[kcycle-adjoint] shape={wl.shape}", flush=True)
    ctx = _ctx(wl, prec="mixed", levels=4)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    g = W.random_vector(wl.shape, 34)
    ref = osolve.direct_solve(p.H2up.conj().T.tocsr(), osolve.rhs_hat(g, wl.tau, wl.omega)).reshape(wl.shape)
    lam, st = ctx.solve_adjoint(_t(g), tol=1e-10, maxit=300)
    assert st["relres"] <= 1e-10
    assert _rel(lam.cpu().numpy(), ref) <= 1e-6


LIMITED = {
    "2d_129_rand_5lv": (lambda: W.random_medium(129, 2, seed=21), 5),
    "3d_65_rand_4lv": (lambda: W.random_medium(65, 3, seed=9), 4),
}


@pytest.mark.parametrize("name", list(LIMITED))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_kcycle_limited_levels(name, prec):
    """The Krylov cycle with the flexible-GMRES coarse solve on level 1 only (V-cycle
    recursion below) against the oracle's cycle with kmax = 1."""
    make, levels = LIMITED[name]
    wl = make()
    print(f"[kcycle-limited] {name} shape={wl.shape} prec={prec}", flush=True)
    ctx = _ctx(wl, prec=prec, levels=levels, kcycle_levels=1)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(levels)
    r = W.random_vector(wl.shape, 81)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    ref = hier.kcycle(r.ravel(), kmax=1).reshape(wl.shape)
    assert _rel(z, ref) <= (1e-10 if prec == "fp64" else 1e-5)
    a, st = ctx.solve(_t(wl.rhs()), tol=1e-8, maxit=500)
    assert st["relres"] <= 1e-8
