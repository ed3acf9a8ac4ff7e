"""Input generators: factored fast marching and the smooth random media (CPU)."""
import numpy as np
import pytest

from paper_1712_06091_amd import workloads as W


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("order", [1, 2])
def test_fast_marching_constant_medium_exact(d, order):
    """tau1 == kappa solves the factored eikonal exactly in a constant medium, and the
    factored update reproduces it (Sec. 1, eq. factoredEikonal)."""
    n = 33 if d == 2 else 17
    shape = (n,) * d
    h = 1.0 / (n - 1)
    src = tuple([n // 2 - 3] + [n // 2 + 1] * (d - 1))
    tau = W.factored_traveltime(np.full(shape, 1.7 ** 2), h, src, order=order)
    np.testing.assert_allclose(tau, 1.7 * W.distance(shape, h, src), rtol=0, atol=1e-12)


def test_fast_marching_linear_gradient_converges():
    """v = 1.5 + 0.8 z against the closed-form first arrival: relative L2 error small and
    the median error falling at second order (second-order one-sided differences)."""
    med, l2 = [], []
    for n in (65, 129):
        wl = W.linear_gradient(n, 2, absorb=False)
        t = W.factored_traveltime(wl.kappa2, wl.h, wl.src, order=2)
        e = np.abs(t - wl.tau)
        med.append(np.median(e))
        l2.append(np.linalg.norm(e) / np.linalg.norm(wl.tau))
    assert l2[-1] < 1e-4
    assert np.log2(med[0] / med[1]) > 1.5


def test_smooth_random_field_recipe():
    f = W.smooth_random_field((65, 65), 1.0 / 64, seed=3)
    g = W.smooth_random_field((65, 65), 1.0 / 64, seed=3)
    assert np.array_equal(f, g)
    assert f.min() >= -1.0 and f.max() <= 1.0
    assert 0.5 < f.std() <= 1.0
    v = W.smooth_random_velocity((65, 65), 1.0 / 64, seed=3)
    assert v.min() >= 1.6 - 1e-12 and v.max() <= 2.4 + 1e-12


def test_random_medium_workload():
    wl = W.random_medium(33, 3, seed=3)
    assert wl.tau[wl.src] == 0.0 and np.all(wl.tau >= 0)
    v_min = np.sqrt(1.0 / wl.kappa2.max())
    assert abs(wl.omega - 2 * np.pi * v_min / (10 * wl.h)) < 1e-9


@pytest.mark.parametrize("n,d,seed", [(129, 3, 3), (65, 3, 7), (257, 2, 4003), (513, 2, 4001)])
def test_fast_marching_random_medium_is_a_first_arrival(n, d, seed):
    """In the smooth random media every node is reached (finite tau), tau >= 0 = tau(source),
    and neighbouring values differ by at most 1.1 h max(kappa_i, kappa_j): a
    first arrival is Lipschitz with the local slowness, so a larger jump is a marching
    error (before the fast marching bounded its factored update this way, 129^3 seed 3
    left 404 nodes unreached and 257^3 seed 3 had jumps of 10 h kappa)."""
    wl = W.random_medium(n, d, seed=seed)
    tau = wl.tau
    assert np.all(np.isfinite(tau))
    assert tau[wl.src] == 0.0 and np.all(tau >= 0)
    kap = np.sqrt(wl.kappa2)
    for ax in range(d):
        t0 = np.take(tau, np.arange(n - 1), axis=ax)
        t1 = np.take(tau, np.arange(1, n), axis=ax)
        k = np.maximum(np.take(kap, np.arange(n - 1), axis=ax), np.take(kap, np.arange(1, n), axis=ax))
        assert np.max(np.abs(t1 - t0) / (wl.h * k)) <= 1.1 * (1 + 1e-12)


def test_batch_workload_parallel_fast_marching_is_identical():
    """The batch recipe with its fast marching in forked workers gives the same shots
    (sizes, sources, media, travel times) as the serial recipe."""
    a = W.batch_2d(count=5, seed=9, sizes=(33, 65))
    b = W.batch_2d(count=5, seed=9, sizes=(33, 65), workers=3)
    for x, y in zip(a, b):
        assert x.shape == y.shape and x.src == y.src and x.omega == y.omega
        assert np.array_equal(x.kappa2, y.kappa2) and np.array_equal(x.tau, y.tau)
        assert np.array_equal(x.gamma, y.gamma)
