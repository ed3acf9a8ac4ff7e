"""GPU parity of the standard Helmholtz path (tau = NULL) and of the shifted-Laplacian
preconditioner (adr_options.shift_alpha), through the C ABI, against the FP64 oracle
(oracle/helmholtz.py).  Every case prints its name and sizes before touching the GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import helmholtz as OH
from oracle import multigrid as omg
from oracle import operators as oops
from oracle import solve as osolve
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
    xs = W.node_coordinates(shape, h)
    v = 1.5 + 0.8 * xs[0]
    omega = W.omega_for_ppw(1.5, h)
    gamma = W.absorbing_layer(shape, h, omega, 4 * h)
    return W.Workload("noncubic", shape, h, omega, (5, 12, 16), 1.0 / v ** 2, np.zeros(shape), gamma)


CASES = {
    "2d_65_const": lambda: W.constant_medium(65, 2),
    "3d_33_lin": lambda: W.linear_gradient(33, 3),
    "3d_noncubic": _noncubic,
}


def _hctx(wl, prec="fp64", alpha=0.2, **opts):
    """A context on the standard Helmholtz operator (tau = NULL)."""
    from paper_1712_06091_amd import adr
    o = adr.default_options(prec=prec, shift_alpha=alpha, **opts)
    gamma = _t(wl.gamma, torch.float64) if wl.gamma is not None else None
    return adr.Context(_t(wl.kappa2, torch.float64), None, gamma, wl.h, wl.omega, wl.src, options=o)


def _oracle(wl, alpha=0.2):
    return OH.HelmholtzProblem(wl.kappa2, wl.gamma, wl.h, wl.omega, alpha=alpha)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("beta", [0.0, 0.25])
def test_apply_is_helmholtz(name, beta):
    """Without tau the fine operator is H for any blend beta (no advection)."""
    wl = CASES[name]()
    print(f"[helm-apply] {name} shape={wl.shape} beta={beta}", flush=True)
    ctx = _hctx(wl)
    p = _oracle(wl)
    g, L, c = ctx.coefficients()
    assert float(torch.abs(g).max()) == 0.0 and float(torch.abs(L).max()) == 0.0
    x = W.random_vector(wl.shape, 21)
    y = ctx.apply(_t(x), beta=beta).cpu().numpy()
    ref = (p.H @ x.ravel()).reshape(wl.shape)
    scale = (abs(p.H) @ np.abs(x.ravel())).reshape(wl.shape)
    assert np.max(np.abs(y - ref) / scale) <= 1e-13


def _stencil_to_csr(planes, offsets, shape):
    d = len(shape)
    st = {}
    for k, (dx, dy, dz) in enumerate(offsets):
        st[(dz, dy, dx)[3 - d:]] = planes[k]
    return oops.stencil_to_csr(st, shape)


@pytest.mark.parametrize("name", list(CASES))
def test_shifted_galerkin_hierarchy(name):
    wl = CASES[name]()
    print(f"[helm-galerkin] {name} shape={wl.shape}", flush=True)
    ctx = _hctx(wl)
    hier = _oracle(wl).hierarchy(ctx.num_levels)
    for l in range(1, ctx.num_levels):
        planes, offs = ctx.level_stencil(l)
        shape, _ = ctx.level_info(l)
        A = _stencil_to_csr(planes.cpu().numpy(), offs, shape)
        err = abs(A - hier.A[l]).max()
        assert err <= 1e-12 * abs(hier.A[l]).max(), (l, err)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("alpha", [0.2, 0.5])
def test_shifted_vcycle_fp64(name, alpha):
    wl = CASES[name]()
    print(f"[helm-vcycle-fp64] {name} shape={wl.shape} alpha={alpha}", flush=True)
    ctx = _hctx(wl, alpha=alpha)
    hier = _oracle(wl, alpha).hierarchy(ctx.num_levels)
    r = W.random_vector(wl.shape, 22)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    assert _rel(z, hier.vcycle(r.ravel()).reshape(wl.shape)) <= 1e-10


@pytest.mark.parametrize("name", ["2d_65_const", "3d_33_lin"])
def test_shifted_kcycle_and_mixed(name):
    wl = CASES[name]()
    print(f"[helm-kcycle] {name} shape={wl.shape}", flush=True)
    r = W.random_vector(wl.shape, 23)
    ctx = _hctx(wl, cycle="k")
    hier = _oracle(wl).hierarchy(ctx.num_levels)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    assert _rel(z, hier.kcycle(r.ravel()).reshape(wl.shape)) <= 1e-10
    ctx32 = _hctx(wl, prec="mixed")
    z32 = ctx32.vcycle(_t(r)).cpu().numpy()
    assert _rel(z32, hier.vcycle(r.ravel()).reshape(wl.shape)) <= 1e-4


def test_shift_on_adr_preconditioner():
    """The shift applies to the ADR preconditioner A_beta too (tau given)."""
    wl = W.linear_gradient(33, 3)
    print(f"[adr-shift] shape={wl.shape}", flush=True)
    from paper_1712_06091_amd import adr
    o = adr.default_options(prec="fp64", shift_alpha=0.3)
    ctx = adr.Context(_t(wl.kappa2, torch.float64), _t(wl.tau, torch.float64), _t(wl.gamma, torch.float64),
                      wl.h, wl.omega, wl.src, options=o)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    As = (p.Abeta - 1j * 0.3 * wl.omega ** 2 * sp.diags(wl.kappa2.ravel())).tocsr()
    hier = omg.Hierarchy(As, wl.shape, ctx.num_levels)
    r = W.random_vector(wl.shape, 24)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    assert _rel(z, hier.vcycle(r.ravel()).reshape(wl.shape)) <= 1e-10
    # the outer operator is still the unshifted H_2up
    x = W.random_vector(wl.shape, 25)
    y = ctx.apply(_t(x), beta=0.0).cpu().numpy()
    assert _rel(y, (p.H2up @ x.ravel()).reshape(wl.shape)) <= 1e-13


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_helmholtz_solve_matches_direct(name, prec):
    wl = CASES[name]()
    print(f"[helm-solve] {name} shape={wl.shape} prec={prec}", flush=True)
    ctx = _hctx(wl, prec=prec)
    p = _oracle(wl)
    q = wl.rhs()
    ref = osolve.direct_solve(p.H, q).reshape(wl.shape)
    u, st = ctx.solve(_t(q), tol=1e-10, maxit=600)
    u = u.cpu().numpy()
    assert st["relres"] <= 1e-10
    assert np.linalg.norm(p.H @ u.ravel() - q.ravel()) / np.linalg.norm(q) <= 2e-10
    assert _rel(u, ref) <= 1e-6
    # tau = 0: the wavefield is the solution itself
    assert np.array_equal(ctx.wavefield(_t(u)).cpu().numpy(), u)


def test_helmholtz_batch_equals_single():
    """Helmholtz shots (tau = NULL) in one batch: each equals its own solve with full
    restart cycles bit for bit."""
    from paper_1712_06091_amd import adr
    wls = [W.constant_medium(65, 2), W.constant_medium(65, 2), W.constant_medium(33, 2)]
    wls[1].src = (20, 40)
    print("[helm-batch] 2d 65, 65, 33", flush=True)
    o = adr.default_options(prec="mixed", shift_alpha=0.2)
    shots = [{"kappa2": _t(w.kappa2, torch.float64), "tau": None, "gamma": _t(w.gamma, torch.float64),
              "h": w.h, "omega": w.omega, "src": w.src} for w in wls]
    qs = [_t(w.rhs(), torch.complex128) for w in wls]
    outs = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in wls]
    b = adr.Batch(shots, options=o, nstreams=2)
    status, stats = b.solve(qs, outs, tol=1e-8, maxit=400)
    assert status == adr.ADR_OK
    b.close()
    o1 = adr.default_options(prec="mixed", shift_alpha=0.2, full_cycles=1)
    for w, q, out in zip(wls, qs, outs):
        ctx = adr.Context(_t(w.kappa2, torch.float64), None, _t(w.gamma, torch.float64), w.h, w.omega, w.src,
                          options=o1)
        a, st = ctx.solve(q, tol=1e-8, maxit=400)
        assert torch.equal(a, out)
        ctx.close()
