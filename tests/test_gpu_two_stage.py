"""GPU parity of the central-advection operator, the H_1up outer operator, the rescaled
(M A M^{-1}) cycle and the two-stage solve of Alg. ADRlong, through the C ABI, against
the FP64 oracle (oracle/two_stage.py).  Every case prints its name before the GPU."""
import numpy as np
import pytest

from oracle import multigrid as omg
from oracle import operators as oops
from oracle import solve as osolve
from oracle import two_stage as ots
from paper_1712_06091_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


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
    gamma = W.absorbing_layer(shape, h, omega, 4 * h)
    return W.Workload("noncubic", shape, h, omega, src, 1.0 / v ** 2, tau, gamma)


CASES = {
    "2d_65_const": lambda: W.constant_medium(65, 2),
    "3d_33_lin": lambda: W.linear_gradient(33, 3),
    "3d_noncubic": _noncubic,
}


def _ctx(wl, options):
    from paper_1712_06091_amd import adr
    return adr.Context(_t(wl.kappa2, torch.float64), _t(wl.tau, torch.float64), _t(wl.gamma, torch.float64),
                       wl.h, wl.omega, wl.src, options=options)


def _opts(prec="fp64", **kw):
    from paper_1712_06091_amd import adr
    return adr.default_options(prec=prec, **kw)


def _oracle(wl):
    return ots.TwoStageProblem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_central_apply(name, beta):
    wl = CASES[name]()
    print(f"[central-apply] {name} shape={wl.shape} beta={beta}", flush=True)
    ctx = _ctx(wl, _opts(advection="central"))
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    A = oops.assemble_adr(p.g, p.L, p.c, wl.h, wl.omega, beta, src=wl.src, central=True)
    x = W.random_vector(wl.shape, 31)
    y = ctx.apply(_t(x), beta=beta).cpu().numpy()
    scale = (abs(A) @ np.abs(x.ravel())).reshape(wl.shape)
    assert np.max(np.abs(y - (A @ x.ravel()).reshape(wl.shape)) / scale) <= 1e-13


@pytest.mark.parametrize("name", ["2d_65_const", "3d_33_lin"])
def test_outer_beta_solves_h1up(name):
    wl = CASES[name]()
    print(f"[h1up-solve] {name} shape={wl.shape}", flush=True)
    ctx = _ctx(wl, _opts(beta=1.0, outer_beta=1.0, cycle="k"))
    p = _oracle(wl)
    qh = osolve.rhs_hat(wl.rhs(), wl.tau, wl.omega)
    a, st = ctx.solve(_t(wl.rhs()), tol=1e-10, maxit=300)
    assert st["relres"] <= 1e-10
    ref = osolve.direct_solve(p.H1up, qh).reshape(wl.shape)
    assert _rel(a.cpu().numpy(), ref) <= 1e-7


def _stage2_opts(prec="fp64", cycle="k"):
    return _opts(prec=prec, advection="central", beta=0.0, shift_alpha=0.2, rescaled=1, cycle=cycle)


def _stencil_to_csr(planes, offsets, shape):
    d = len(shape)
    st = {}
    for k, (dx, dy, dz) in enumerate(offsets):
        st[(dz, dy, dx)[3 - d:]] = planes[k]
    return oops.stencil_to_csr(st, shape)


@pytest.mark.parametrize("name", list(CASES))
def test_rescaled_galerkin_hierarchy(name):
    """Coarse levels of the second stage are Galerkin products of the shifted rescaled
    operator M H_cen M^{-1} - i w^2 alpha diag(kappa^2)."""
    wl = CASES[name]()
    print(f"[rescaled-galerkin] {name} shape={wl.shape}", flush=True)
    ctx = _ctx(wl, _stage2_opts())
    hier = omg.Hierarchy(_oracle(wl).Bs, wl.shape, ctx.num_levels)
    for l in range(1, ctx.num_levels):
        planes, offs = ctx.level_stencil(l)
        shape, _ = ctx.level_info(l)
        A = _stencil_to_csr(planes.cpu().numpy(), offs, shape)
        err = abs(A - hier.A[l]).max()
        assert err <= 1e-12 * abs(hier.A[l]).max(), (l, err)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("cycle", ["v", "k"])
def test_rescaled_cycle(name, cycle):
    """The library's cycle (in a) is M^{-1} K(M r), K the oracle's cycle on the shifted
    rescaled operator (in u)."""
    wl = CASES[name]()
    print(f"[rescaled-cycle] {name} shape={wl.shape} cycle={cycle}", flush=True)
    ctx = _ctx(wl, _stage2_opts(cycle=cycle))
    p = _oracle(wl)
    hier = omg.Hierarchy(p.Bs, wl.shape, ctx.num_levels)
    r = W.random_vector(wl.shape, 32).ravel()
    K = hier.vcycle if cycle == "v" else hier.kcycle
    ref = (K(p.m * r) / p.m).reshape(wl.shape)
    z = ctx.vcycle(_t(r.reshape(wl.shape))).cpu().numpy()
    assert _rel(z, ref) <= 1e-10
    if cycle == "v":
        ctx32 = _ctx(wl, _stage2_opts(prec="mixed", cycle=cycle))
        z32 = ctx32.vcycle(_t(r.reshape(wl.shape))).cpu().numpy()
        assert _rel(z32, ref) <= 1e-4


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_two_stage_solve(name, prec):
    from paper_1712_06091_amd import adr
    wl = CASES[name]()
    print(f"[two-stage] {name} shape={wl.shape} prec={prec}", flush=True)
    o1, o2 = adr.two_stage_options(prec)
    assert o2.rescaled == 1 and o2.advection == adr.ADR_ADV_CENTRAL and o1.outer_beta == 1.0
    c1, c2 = _ctx(wl, o1), _ctx(wl, o2)
    p = _oracle(wl)
    q = wl.rhs()
    a, s1, s2 = adr.solve_two_stage(c1, c2, _t(q), tol=1e-10, maxit=400)
    assert s2["status"] == adr.ADR_OK and s2["relres"] <= 1e-10
    assert s1["outer_iters"] <= 5
    qh = osolve.rhs_hat(q, wl.tau, wl.omega)
    ref = osolve.direct_solve(p.Hcen, qh).reshape(wl.shape)
    a = a.cpu().numpy()
    assert np.linalg.norm(p.Hcen @ a.ravel() - qh.ravel()) / np.linalg.norm(qh) <= 2e-10
    assert _rel(a, ref) <= 1e-6
    if prec == "fp64":
        # the first stage alone equals the oracle's first stage
        a1, st1 = c1.solve(_t(q), tol=1e-2, maxit=5)
        o_a1, info1 = p.stage1(qh.ravel())
        assert st1["outer_iters"] == info1["iters"] == s1["outer_iters"]
        assert _rel(a1.cpu().numpy(), o_a1.reshape(wl.shape)) <= 1e-9


def test_two_stage_without_first_stage_and_bad_pairs():
    """maxit_first = 0 leaves a = 0 after stage 1, so the result is stage 2's solve from
    zero; contexts on different grids are refused."""
    from paper_1712_06091_amd import adr
    wl = W.constant_medium(65, 2)
    print("[two-stage-edge] 2d 65", flush=True)
    o1, o2 = adr.two_stage_options("fp64")
    c1, c2 = _ctx(wl, o1), _ctx(wl, o2)
    q = _t(wl.rhs())
    a, s1, s2 = adr.solve_two_stage(c1, c2, q, tol=1e-10, maxit=400, maxit_first=0)
    assert s1["outer_iters"] == 0 and s2["relres"] <= 1e-10
    b, st = c2.solve(q, tol=1e-10, maxit=400)
    assert st["outer_iters"] == s2["outer_iters"]
    assert _rel(a.cpu().numpy(), b.cpu().numpy()) <= 1e-12
    other = W.constant_medium(33, 2)
    c3 = _ctx(other, o2)
    with pytest.raises(adr.AdrError) as e:
        adr.solve_two_stage(c1, c3, q, tol=1e-10, maxit=10)
    assert e.value.status == adr.ADR_EINVAL


def test_rescaled_refuses_adjoint_and_batch():
    from paper_1712_06091_amd import adr
    wl = W.constant_medium(33, 2)
    print("[rescaled-refuse] 2d 33", flush=True)
    ctx = _ctx(wl, _stage2_opts())
    with pytest.raises(adr.AdrError) as e:
        ctx.solve_adjoint(_t(wl.rhs()), tol=1e-6, maxit=10)
    assert e.value.status == adr.ADR_ENOTSUP
    shot = {"kappa2": _t(wl.kappa2, torch.float64), "tau": _t(wl.tau, torch.float64),
            "gamma": _t(wl.gamma, torch.float64), "h": wl.h, "omega": wl.omega, "src": wl.src}
    with pytest.raises(adr.AdrError) as e:
        adr.Batch([shot, shot], options=_stage2_opts())
    assert e.value.status == adr.ADR_ENOTSUP
