"""The LDS z-marching tiles of the matrix-free finest level (Jacobi sweeps and the V-cycle
residual) do the one-lane kernels' arithmetic: cycles and whole solves are bit-identical
with and without them, on cubic, non-cubic and shot-group launches, and match the oracle."""
import numpy as np
import pytest

from oracle import solve as osolve
from paper_1712_06091_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _noncubic():
    shape = (17, 25, 33)
    h = 1.0 / 32
    src = (5, 12, 16)
    xs = W.node_coordinates(shape, h)
    v = 1.5 + 0.8 * xs[0]
    tau = W.linear_velocity_traveltime(shape, h, src, 1.5, 0.8)
    omega = W.omega_for_ppw(1.5, h)
    return W.Workload("noncubic", shape, h, omega, src, 1.0 / v ** 2, tau, W.absorbing_layer(shape, h, omega, 4 * h))


CASES = {
    "3d_65_rand": lambda: W.random_medium(65, 3, seed=9),
    "3d_129_lin": lambda: W.linear_gradient(129, 3),
    "3d_noncubic": _noncubic,
}


def _ctx(wl, tiles, **kw):
    from paper_1712_06091_amd import adr
    return adr.Context(_t(wl.kappa2, torch.float64), _t(wl.tau, torch.float64), _t(wl.gamma, torch.float64),
                       wl.h, wl.omega, wl.src, options=adr.default_options(prec="mixed", fine_tiles=tiles, **kw))


@pytest.mark.parametrize("name", list(CASES))
def test_fine_tiles_bit_identical(name):
    wl = CASES[name]()
    print(f"[fine-tiles] {name} shape={wl.shape}", flush=True)
    on, off = _ctx(wl, 2), _ctx(wl, 0)
    r = _t(W.random_vector(wl.shape, 91))
    z1, z0 = on.vcycle(r), off.vcycle(r)
    assert torch.equal(z1, z0)
    q = _t(wl.rhs())
    a1, s1 = on.solve(q, tol=1e-8, maxit=400)
    a0, s0 = off.solve(q, tol=1e-8, maxit=400)
    assert s1["outer_iters"] == s0["outer_iters"] and torch.equal(a1, a0)
    if wl.nodes <= 300000:
        p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
        hier = p.hierarchy(on.num_levels)
        ref = hier.vcycle(r.cpu().numpy().ravel()).reshape(wl.shape)
        zz = z1.cpu().numpy()
        assert np.linalg.norm(zz - ref) / np.linalg.norm(ref) <= 1e-5
    on.close()
    off.close()


def test_fine_tiles_in_shot_groups():
    """Shot groups of a 3D shape take the tiles too; per shot the batch equals single
    solves with full restart cycles bit for bit."""
    from paper_1712_06091_amd import adr
    wls = [W.random_medium(33, 3, seed=s) for s in (61, 62)]
    print("[fine-tiles-batch] 2 shots 33^3", flush=True)
    shots = [{"kappa2": _t(w.kappa2, torch.float64), "tau": _t(w.tau, torch.float64),
              "gamma": _t(w.gamma, torch.float64), "h": w.h, "omega": w.omega, "src": w.src} for w in wls]
    qs = [_t(w.rhs(), torch.complex128) for w in wls]
    outs = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in wls]
    b = adr.Batch(shots, options=adr.default_options(prec="mixed", fine_tiles=2), nstreams=1)
    st, stats = b.solve(qs, outs, tol=1e-8, maxit=400)
    assert st == adr.ADR_OK
    for i, w in enumerate(wls):
        c = _ctx(w, 0, full_cycles=1)
        a, s1 = c.solve(qs[i], tol=1e-8, maxit=400)
        assert s1["outer_iters"] == stats[i]["outer_iters"] and torch.equal(a, outs[i]), i
        c.close()
    b.close()
