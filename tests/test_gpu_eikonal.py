"""GPU factored-eikonal sweeps (adr_eikonal) against the oracle's sweeps: same fixed point
node for node, same number of sweeps, on 2D/3D, random and smooth media, non-cubic grids
and sources next to a face or in a corner; plus the error paths."""
import numpy as np
import pytest

from oracle import eikonal as oeik
from paper_1712_06091_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _noncubic():
    shape = (17, 25, 33)
    h = 1.0 / 32
    xs = W.node_coordinates(shape, h)
    v = 1.5 + 0.8 * xs[0]
    return 1.0 / v ** 2, h, (2, 12, 30)


CASES = {
    "2d_129_rand": lambda: (lambda w: (w.kappa2, w.h, w.src))(W.random_medium(129, 2, seed=4001)),
    "3d_33_lin": lambda: (lambda w: (w.kappa2, w.h, w.src))(W.linear_gradient(33, 3)),
    "3d_65_rand": lambda: (lambda w: (w.kappa2, w.h, w.src))(W.random_medium(65, 3, seed=9)),
    "3d_noncubic_face": _noncubic,
    "2d_corner": lambda: (1.0 / (2.0 + np.arange(7 * 9).reshape(7, 9) % 5 * 0.1) ** 2, 0.125, (0, 0)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_eikonal_matches_oracle(name):
    from paper_1712_06091_amd import adr
    kappa2, h, src = CASES[name]()
    print(f"[eikonal] {name} shape={kappa2.shape} src={src}", flush=True)
    tau, sweeps = adr.eikonal(_t(kappa2), h, src)
    tau = tau.cpu().numpy()
    ref, ref_sweeps = oeik.factored_eikonal(kappa2, h, src)
    assert np.all(np.isfinite(tau)) and tau[tuple(src)] == 0.0
    err = np.max(np.abs(tau - ref)) / np.max(ref)
    print(f"[eikonal] sweeps gpu {sweeps} oracle {ref_sweeps}, max rel diff {err:.1e}", flush=True)
    assert err <= 1e-12
    assert sweeps == ref_sweeps


def test_eikonal_constant_medium_exact_and_errors():
    from paper_1712_06091_amd import adr
    shape = (33, 33, 33)
    h = 1.0 / 32
    src = (10, 17, 20)
    print("[eikonal] constant 33^3 and error paths", flush=True)
    tau, _ = adr.eikonal(_t(np.full(shape, 0.49)), h, src)
    np.testing.assert_allclose(tau.cpu().numpy(), 0.7 * W.distance(shape, h, src), rtol=0, atol=1e-12)
    with pytest.raises(adr.AdrError) as err:
        adr.eikonal(_t(np.full(shape, 0.49)), h, (40, 0, 0))
    assert err.value.status == adr.ADR_EINVAL
    # too few sweeps: ENOCONV is a status the binding passes through; the iterate is partial
    kappa2 = _t(np.full(shape, 0.49))
    import ctypes
    lib = adr.load_library()
    n = (ctypes.c_int * 3)(33, 33, 33)
    s = (ctypes.c_int * 3)(src[2], src[1], src[0])
    out = torch.empty_like(kappa2)
    work = torch.empty(kappa2.numel() + 1, dtype=torch.float64, device="cuda")
    sw = ctypes.c_int()
    st = lib.adr_eikonal(3, n, h, adr._dev(kappa2, torch.float64), s, adr._dev(out, torch.float64),
                         adr._dev(work, torch.float64), 3, ctypes.byref(sw), None)
    assert st == adr.ADR_ENOCONV and sw.value == 3


def test_eikonal_full_size_fixed_point():
    """At the 3D 129^3 random-medium size (sweeps of the oracle to the end would take
    minutes): the GPU result is a fixed point of the oracle's sweep, finite, zero at the
    source and Lipschitz with the local slowness."""
    from paper_1712_06091_amd import adr
    n = 129
    shape = (n,) * 3
    h = 1.0 / (n - 1)
    kappa2 = 1.0 / W.smooth_random_velocity(shape, h, 24) ** 2
    src = (13, 64, 64)
    print("[eikonal] 129^3 random medium, fixed point of the oracle sweep", flush=True)
    tau, sweeps = adr.eikonal(_t(kappa2), h, src)
    tau = tau.cpu().numpy()
    assert np.all(np.isfinite(tau)) and tau[src] == 0.0
    assert np.array_equal(oeik.sweep(tau, kappa2, h, src), tau)
    kap = np.sqrt(kappa2)
    for ax in range(3):
        dt = np.abs(np.diff(tau, axis=ax))
        k = np.maximum(np.take(kap, np.arange(n - 1), axis=ax), np.take(kap, np.arange(1, n), axis=ax))
        assert np.max(dt / (h * k)) <= 1.1 * (1 + 1e-12)
