"""Seeded synthetic inputs for the ADR-amplitude solve: media, travel times, absorbing
layers, sources.  Shared by the tests, the benchmark and the smoke check.

This module holds none of the solver's arithmetic: it only builds the inputs that the
solver takes (kappa^2, tau, gamma, the source node and the point-source right-hand side).
The paper's own performance media (a figure-only linear model, Marmousi2, Overthrust)
are not available, so these synthetic media stand in for them with the paper's kind of
setting (Sec. 4.2): smooth velocity, about 10 points per wavelength, a point source in
the interior of a unit square / cube.

Arrays are C-ordered with the last axis = x (fastest); axis 0 is depth (y in 2D, z in
3D).  Source indices are NumPy index tuples in the same order.
"""
import ctypes
import os
import time
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np


@dataclass
class Workload:
    name: str
    shape: Tuple[int, ...]
    h: float
    omega: float
    src: Tuple[int, ...]
    kappa2: np.ndarray
    tau: np.ndarray
    gamma: Optional[np.ndarray]
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def nodes(self):
        return int(np.prod(self.shape))

    def rhs(self):
        """Point source q = e_src / h^d (Sec. 4.1 discretizes delta as 1/h^d)."""
        q = np.zeros(self.shape, dtype=np.complex128)
        q[self.src] = 1.0 / self.h ** self.ndim
        return q


def node_coordinates(shape, h):
    return np.meshgrid(*[np.arange(n, dtype=np.float64) * h for n in shape], indexing="ij")


def distance(shape, h, src):
    xs = node_coordinates(shape, h)
    return np.sqrt(sum((x - s * h) ** 2 for x, s in zip(xs, src)))


def omega_for_ppw(v_min, h, ppw=10.0):
    """Angular frequency giving ``ppw`` nodes per minimum wavelength v_min / f."""
    return 2.0 * np.pi * v_min / (ppw * h)


def absorbing_layer(shape, h, omega, thickness, faces=None):
    """gamma rising quadratically from 0 to omega over ``thickness`` towards the listed
    faces (Sec. 1); in several dimensions the largest per-axis value.  ``faces`` is a
    list of (axis, side) with side 0 = low, 1 = high; default: every face."""
    d = len(shape)
    if faces is None:
        faces = [(a, s) for a in range(d) for s in (0, 1)]
    xs = node_coordinates(shape, h)
    gam = np.zeros(shape)
    for a, side in faces:
        extent = (shape[a] - 1) * h
        depth = xs[a] if side == 0 else extent - xs[a]
        pen = np.clip((thickness - depth) / thickness, 0.0, 1.0)
        gam = np.maximum(gam, omega * pen ** 2)
    return gam


def linear_velocity_traveltime(shape, h, src, v0, grad):
    """First-arrival time for v = v0 + grad * depth (depth = axis 0) from node ``src``:
    tau = (1/g) arccosh(1 + g^2 |x - x0|^2 / (2 v(x) v(x0)))."""
    xs = node_coordinates(shape, h)
    depth = xs[0]
    v = v0 + grad * depth
    v_src = v0 + grad * src[0] * h
    r2 = sum((x - s * h) ** 2 for x, s in zip(xs, src))
    if grad == 0.0:
        return np.sqrt(r2) / v0
    return np.arccosh(1.0 + grad * grad * r2 / (2.0 * v * v_src)) / grad


def constant_medium(n, ndim=2, ppw=10.0, absorb=True, src=None, name="const"):
    """kappa = 1 on the unit square/cube, tau = r, source at the centre node."""
    shape = (n,) * ndim
    h = 1.0 / (n - 1)
    omega = omega_for_ppw(1.0, h, ppw)
    src = tuple(s for s in (src if src is not None else (n // 2,) * ndim))
    kappa2 = np.ones(shape)
    tau = distance(shape, h, src)
    gamma = absorbing_layer(shape, h, omega, 10 * h) if absorb else None
    return Workload(name, shape, h, omega, src, kappa2, tau, gamma)


def linear_gradient(n, ndim=3, v0=1.5, grad=0.8, ppw=10.0, src_frac=None, absorb=True,
                    name="linear_gradient"):
    """v = v0 + grad*depth over the unit square/cube, analytic tau, source at
    (0.5, 0.5, 0.1) (depth fraction last in ``src_frac`` order x, y, depth) snapped to
    the nearest node."""
    shape = (n,) * ndim
    h = 1.0 / (n - 1)
    if src_frac is None:
        src_frac = (0.5,) * (ndim - 1) + (0.1,)
    # src_frac is (x, y, ..., depth); NumPy order is (depth, ..., y, x).
    src = tuple(int(round(f / h)) for f in reversed(src_frac))
    v = v0 + grad * node_coordinates(shape, h)[0]
    kappa2 = 1.0 / v ** 2
    tau = linear_velocity_traveltime(shape, h, src, v0, grad)
    omega = omega_for_ppw(v0, h, ppw)
    gamma = absorbing_layer(shape, h, omega, 10 * h) if absorb else None
    return Workload(name, shape, h, omega, src, kappa2, tau, gamma)


def config_2d_129():
    """2D 129^2 unit square, kappa = 1, 10 points per wavelength, source (0.5, 0.5)."""
    return constant_medium(129, ndim=2, name="2d_129_const")


def config_3d_129():
    """3D 129^3 unit cube (1 km), v = 1.5 + 0.8 z km/s, analytic tau, source
    (0.5, 0.5, 0.1) km snapped to node (x, y, z) = (64, 64, 13), 10 points per
    wavelength at v_min = 1.5 km/s."""
    return linear_gradient(129, ndim=3, name="3d_129_linear_gradient")


def random_vector(shape, seed, dtype=np.complex128):
    """Seeded complex Gaussian test vector."""
    rng = np.random.default_rng(seed)
    if np.dtype(dtype).kind == "c":
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)
    return rng.standard_normal(shape).astype(dtype)


# ---------------------------------------------------------------------------------------
# Random media and fast-marching travel times (configurations with heterogeneous media)
# ---------------------------------------------------------------------------------------
def smooth_random_field(shape, h, seed, corr_len=0.1):
    """eta = G_sigma * xi, xi iid N(0, 1) (seeded), sigma = corr_len in domain units (a
    periodic Gaussian filter applied in Fourier space), normalized to unit standard
    deviation, then clipped to [-1, 1]."""
    from scipy.ndimage import fourier_gaussian
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(shape)
    axes = tuple(range(len(shape)))
    eta = np.fft.irfftn(fourier_gaussian(np.fft.rfftn(xi), sigma=corr_len / h, n=shape[-1]), s=shape, axes=axes)
    eta = eta / eta.std()
    return np.clip(eta, -1.0, 1.0)


def smooth_random_velocity(shape, h, seed, v0=2.0, amp=0.2, corr_len=0.1):
    """v = v0 (1 + amp * eta) km/s (eta from smooth_random_field)."""
    return v0 * (1.0 + amp * smooth_random_field(shape, h, seed, corr_len))


_fm = None


def _fm_lib():
    global _fm
    if _fm is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfm.so")
        if not os.path.exists(path):
            raise RuntimeError("libfm.so not built (run __graft_entry__.build())")
        lib = ctypes.CDLL(path)
        lib.fm_factored.restype = ctypes.c_int
        lib.fm_factored.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_double, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_void_p]
        _fm = lib
    return _fm


def factored_traveltime(kappa2, h, src, order=2):
    """First-arrival travel time from node ``src`` (NumPy index order) by factored fast
    marching (CPU, libfm.so)."""
    kappa2 = np.ascontiguousarray(kappa2, dtype=np.float64)
    d = kappa2.ndim
    n = (ctypes.c_int * 3)(*[kappa2.shape[d - 1 - k] if k < d else 1 for k in range(3)])
    s = (ctypes.c_int * 3)(*[int(src[d - 1 - k]) if k < d else 0 for k in range(3)])
    tau = np.empty_like(kappa2)
    rc = _fm_lib().fm_factored(d, n, float(h), kappa2.ctypes.data, s, int(order), tau.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"fast marching failed ({rc})")
    return tau


def random_medium(n, ndim, seed, src_frac=None, ppw=10.0, absorb=True, name="random_medium", order=2):
    """Unit square/cube, v = 2 (1 + 0.2 eta) km/s with eta seeded and smoothed over 0.1 km,
    tau by factored fast marching, 10 points per wavelength at the slowest velocity."""
    shape = (n,) * ndim
    h = 1.0 / (n - 1)
    if src_frac is None:
        src_frac = (0.5,) * (ndim - 1) + (0.1,)
    src = tuple(int(round(f / h)) for f in reversed(src_frac))
    v = smooth_random_velocity(shape, h, seed)
    kappa2 = 1.0 / v ** 2
    t0 = time.perf_counter()
    tau = factored_traveltime(kappa2, h, src, order=order)
    fm_s = time.perf_counter() - t0
    omega = omega_for_ppw(float(v.min()), h, ppw)
    gamma = absorbing_layer(shape, h, omega, 10 * h) if absorb else None
    return Workload(name, shape, h, omega, src, kappa2, tau, gamma, extra={"seed": seed, "fm_s": fm_s})


def config_3d_257():
    """3D 257^3 unit cube, v = 2 (1 + 0.2 eta) km/s (seed 3), tau by factored fast
    marching, source (0.5, 0.5, 0.1) km, 10 points per wavelength."""
    return random_medium(257, 3, seed=3, name="3d_257_random")


def batch_2d(count=64, seed=4, sizes=(257, 513, 1025), margin=12, name="batch_2d", workers=1):
    """``count`` 2D shots on the unit square: grid sizes drawn uniformly from ``sizes``
    and source nodes uniformly at least ``margin`` nodes from the faces (both seeded by
    ``seed``), medium v = 2 (1 + 0.2 eta) with eta seeded by 1000*seed + i, tau by factored
    fast marching, 10 points per wavelength per shot.  ``workers`` > 1 runs the fast
    marching in a pool of forked processes (call it before the GPU is initialized)."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    media = []
    for i, n in enumerate(ns):
        n = int(n)
        h = 1.0 / (n - 1)
        src = tuple(int(v) for v in rng.integers(margin, n - margin, size=2))
        v = smooth_random_velocity((n, n), h, 1000 * seed + i)
        media.append((n, h, src, v))
    jobs = [(1.0 / v ** 2, h, src) for n, h, src, v in media]
    if workers > 1 and count > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, count)) as pool:
            taus = pool.map(_fm_worker, jobs)
    else:
        taus = [_fm_worker(j) for j in jobs]
    shots = []
    for i, ((n, h, src, v), (kappa2, _, _), tau) in enumerate(zip(media, jobs, taus)):
        omega = omega_for_ppw(float(v.min()), h)
        gamma = absorbing_layer((n, n), h, omega, 10 * h)
        shots.append(Workload(f"{name}_{i}", (n, n), h, omega, src, kappa2, tau, gamma, extra={"seed": 1000 * seed + i}))
    return shots


def _fm_worker(args):
    kappa2, h, src = args
    return factored_traveltime(kappa2, h, src)


def factored_traveltimes(kappa2, h, sources, workers=8):
    """Fast-marching travel times for several sources in a pool of forked CPU processes
    (each source is independent).  Call it before the process initializes the GPU."""
    import multiprocessing as mp
    if workers <= 1 or len(sources) <= 1:
        return [factored_traveltime(kappa2, h, s) for s in sources]
    with mp.get_context("fork").Pool(min(workers, len(sources))) as pool:
        return pool.map(_fm_worker, [(kappa2, h, s) for s in sources])


@dataclass
class AdjointWorkload:
    name: str
    shape: Tuple[int, ...]
    h: float
    omega: float
    kappa2: np.ndarray          # model at which the gradient is taken
    kappa2_true: np.ndarray     # model that produced the observed data
    gamma: np.ndarray
    sources: list               # NumPy-order node tuples
    taus: list                  # travel times in kappa2 (held fixed)
    receivers: np.ndarray       # int32 linear node indices


def adjoint_3d(n=193, seed=5, nsrc_axis=4, nrec_axis=64, pert=0.05, eta_seed=55, rec_first=2, rec_step=3,
               workers=8, name=None):
    """3D n^3 unit cube, v = 2 (1 + 0.2 eta) km/s (seed), nsrc_axis^2 sources on a regular
    grid at depth 0.1 km (x, y in {1, ..., nsrc_axis} / (nsrc_axis + 1) km), an
    nrec_axis^2 receiver plane on the top face (z = 0) at nodes i, j = rec_first + rec_step k,
    k = 0 .. nrec_axis - 1, observed data from kappa2_true = kappa2 (1 + pert * eta2) with
    eta2 a smooth field seeded by eta_seed, tau by factored fast marching in kappa2, 10
    points per wavelength."""
    shape = (n,) * 3
    h = 1.0 / (n - 1)
    last = rec_first + rec_step * (nrec_axis - 1)
    if last >= n:
        raise ValueError(f"receiver line {rec_first} + {rec_step} k, k < {nrec_axis}, leaves a grid of {n} nodes")
    v = smooth_random_velocity(shape, h, seed)
    kappa2 = 1.0 / v ** 2
    kappa2_true = kappa2 * (1.0 + pert * smooth_random_field(shape, h, eta_seed))
    omega = omega_for_ppw(float(v.min()), h)
    gamma = absorbing_layer(shape, h, omega, 10 * h)
    fr = [(k + 1) / (nsrc_axis + 1) for k in range(nsrc_axis)]
    sources = [(int(round(0.1 / h)), int(round(y / h)), int(round(x / h))) for y in fr for x in fr]
    taus = factored_traveltimes(kappa2, h, sources, workers)
    line = rec_first + rec_step * np.arange(nrec_axis, dtype=np.int64)
    yy, xx = np.meshgrid(line, line, indexing="ij")
    receivers = np.ravel_multi_index((np.zeros(yy.size, dtype=np.int64), yy.ravel(), xx.ravel()), shape)
    return AdjointWorkload(name or f"adjoint_3d_{n}", shape, h, omega, kappa2, kappa2_true, gamma, sources, taus,
                           receivers.astype(np.int32))
