"""GPU parity of the paper's relaxation on every level (Sec. 4.2): Jacobi-preconditioned
GMRES on the matrix-free finest level as well as on the Galerkin levels, in the V-cycle
and the Krylov cycle, single solves and shot groups, against the oracle's cycles with
GMRES relaxation everywhere."""
import numpy as np
import pytest

from oracle import solve as osolve
from paper_1712_06091_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "2d_65_const": lambda: W.constant_medium(65, 2),
    "3d_33_lin": lambda: W.linear_gradient(33, 3),
    "3d_65_rand": lambda: W.random_medium(65, 3, seed=9),
}


def _t(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _opts(prec, **kw):
    from paper_1712_06091_amd import adr
    return adr.default_options(prec=prec, relax=[adr.ADR_RELAX_GMRES] * 8, **kw)


def _ctx(wl, prec, **kw):
    from paper_1712_06091_amd import adr
    return adr.Context(_t(wl.kappa2, torch.float64), _t(wl.tau, torch.float64), _t(wl.gamma, torch.float64),
                       wl.h, wl.omega, wl.src, options=_opts(prec, **kw))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("cycle", ["v", "k"])
def test_cycle_fine_gmres_fp64(name, cycle):
    wl = CASES[name]()
    print(f"[fine-gmres] {name} shape={wl.shape} cycle={cycle} fp64", flush=True)
    ctx = _ctx(wl, "fp64", cycle=cycle)
    levels = ctx.num_levels
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(levels, smoothers=["gmres"] * levels)
    r = W.random_vector(wl.shape, 71)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    ctx.close()
    ref = (hier.vcycle(r.ravel()) if cycle == "v" else hier.kcycle(r.ravel())).reshape(wl.shape)
    assert _rel(z, ref) <= 1e-10


@pytest.mark.parametrize("name", ["2d_65_const", "3d_65_rand"])
def test_cycle_fine_gmres_mixed(name):
    wl = CASES[name]()
    print(f"[fine-gmres] {name} shape={wl.shape} mixed", flush=True)
    ctx = _ctx(wl, "mixed")
    levels = ctx.num_levels
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(levels, smoothers=["gmres"] * levels)
    r = W.random_vector(wl.shape, 72)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    ctx.close()
    assert _rel(z, hier.vcycle(r.ravel()).reshape(wl.shape)) <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_fine_gmres(prec):
    """Whole solve with GMRES relaxation on every level: the oracle's direct solution to
    1e-6 at tol 1e-10, true residual by the oracle's H_2up."""
    wl = CASES["3d_33_lin"]()
    print(f"[fine-gmres-solve] 3d 33 prec={prec}", flush=True)
    ctx = _ctx(wl, prec)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    qh = osolve.rhs_hat(wl.rhs(), wl.tau, wl.omega)
    ref = osolve.direct_solve(p.H2up, qh).reshape(wl.shape)
    a, st = ctx.solve(_t(wl.rhs()), tol=1e-10, maxit=400)
    a = a.cpu().numpy()
    assert st["relres"] <= 1e-10
    assert np.linalg.norm(p.H2up @ a.ravel() - qh.ravel()) / np.linalg.norm(qh) <= 2e-10
    assert _rel(a, ref) <= 1e-6
    # the adjoint of this cycle is not offered
    from paper_1712_06091_amd import adr
    with pytest.raises(adr.AdrError) as err:
        ctx.solve_adjoint(_t(wl.rhs()), tol=1e-8, maxit=10)
    assert err.value.status == adr.ADR_ENOTSUP
    ctx.close()


def test_batch_fine_gmres_matches_single():
    """Shot groups with GMRES relaxation on the finest level equal single solves with full
    restart cycles bit for bit."""
    from paper_1712_06091_amd import adr
    wls = [W.random_medium(65, 2, seed=s) for s in (51, 52)] + [W.constant_medium(33, 2)]
    print(f"[fine-gmres-batch] {len(wls)} shots", flush=True)
    shots = [{"kappa2": _t(w.kappa2, torch.float64), "tau": _t(w.tau, torch.float64),
              "gamma": _t(w.gamma, torch.float64), "h": w.h, "omega": w.omega, "src": w.src} for w in wls]
    qs = [_t(w.rhs(), torch.complex128) for w in wls]
    outs = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in wls]
    b = adr.Batch(shots, options=_opts("mixed"), nstreams=2)
    st, stats = b.solve(qs, outs, tol=1e-8, maxit=400)
    assert st == adr.ADR_OK
    for i, w in enumerate(wls):
        c = adr.Context(shots[i]["kappa2"], shots[i]["tau"], shots[i]["gamma"], w.h, w.omega, w.src,
                        options=_opts("mixed", full_cycles=1))
        a, s1 = c.solve(qs[i], tol=1e-8, maxit=400)
        assert s1["outer_iters"] == stats[i]["outer_iters"], i
        assert torch.equal(a, outs[i]), i
        c.close()
    b.close()
