"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Every case prints its name and sizes before touching the GPU.  Sizes span several
blocks with ragged tails (N not a multiple of 256) and non-cubic grids.
"""
import numpy as np
import pytest

from oracle import coefficients as ocoef
from oracle import multigrid as omg
from oracle import operators as oops
from oracle import solve as osolve
from paper_1712_06091_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _ctx(wl, prec="fp64", factored=True, **opts):
    from paper_1712_06091_amd import adr
    o = adr.default_options(prec=prec, **opts)
    gamma = _t(wl.gamma, torch.float64) if wl.gamma is not None else None
    return adr.Context(_t(wl.kappa2, torch.float64), _t(wl.tau, torch.float64), gamma, wl.h, wl.omega,
                       wl.src if factored else None, options=o, factored=factored)


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _noncubic():
    """3D 17 x 25 x 33 (z, y, x) linear-gradient medium, source at (z, y, x) = (5, 12, 16)."""
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


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("factored", [True, False])
def test_coefficients(name, factored):
    wl = CASES[name]()
    print(f"[coef] {name} shape={wl.shape} factored={factored}", flush=True)
    ctx = _ctx(wl, factored=factored)
    g, L, c = ctx.coefficients()
    og, oL, oc = ocoef.adr_coefficients(wl.tau, wl.kappa2, wl.gamma, wl.h, wl.omega,
                                        src=wl.src if factored else None)
    d = wl.ndim
    for k in range(d):   # ABI axis k = NumPy axis d-1-k
        ref = og[d - 1 - k]
        assert np.max(np.abs(g[k].cpu().numpy() - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())
    assert np.max(np.abs(L.cpu().numpy() - oL)) <= 1e-12 * np.abs(oL).max()
    assert np.max(np.abs(c.cpu().numpy() - oc)) <= 1e-11 * max(np.abs(oc).max(), wl.omega ** 2)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("beta", [0.0, 0.25, 1.0])
def test_apply(name, beta):
    wl = CASES[name]()
    print(f"[apply] {name} shape={wl.shape} beta={beta}", flush=True)
    ctx = _ctx(wl)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src, beta=beta)
    x = W.random_vector(wl.shape, 11)
    y = ctx.apply(_t(x), beta=beta).cpu().numpy()
    ref = (p.Abeta @ x.ravel()).reshape(wl.shape)
    # Entry-wise bound: rounding of each row's sum, relative to sum_j |A_ij x_j|.
    scale = (abs(p.Abeta) @ np.abs(x.ravel())).reshape(wl.shape)
    assert np.max(np.abs(y - ref) / scale) <= 1e-13


def test_apply_unfactored_plane_wave():
    """src[0] < 0 path (plain differences of tau, no near-source rule)."""
    wl = W.constant_medium(33, 3)
    xs = W.node_coordinates(wl.shape, wl.h)
    tau = 0.6 * xs[2] + 0.8 * xs[0]
    wl.tau = tau
    print("[apply-unfactored] 3d 33", flush=True)
    ctx = _ctx(wl, factored=False)
    g, L, c = ocoef.adr_coefficients(tau, wl.kappa2, wl.gamma, wl.h, wl.omega, src=None)
    A = oops.assemble_adr(g, L, c, wl.h, wl.omega, 0.0, src=None)
    x = W.random_vector(wl.shape, 12)
    y = ctx.apply(_t(x), beta=0.0).cpu().numpy()
    scale = (abs(A) @ np.abs(x.ravel())).reshape(wl.shape)
    assert np.max(np.abs(y - (A @ x.ravel()).reshape(wl.shape)) / scale) <= 1e-13


def _stencil_to_csr(planes, offsets, shape):
    """Assemble GPU planes (S, *shape) with (dx, dy, dz) offsets into a CSR matrix."""
    d = len(shape)
    st = {}
    for p, (dx, dy, dz) in enumerate(offsets):
        key = (dz, dy, dx)[3 - d:]
        st[key] = planes[p]
    return oops.stencil_to_csr(st, shape)


@pytest.mark.parametrize("name", ["2d_65_const", "3d_33_lin", "3d_noncubic"])
def test_galerkin_hierarchy(name):
    wl = CASES[name]()
    print(f"[galerkin] {name} shape={wl.shape}", flush=True)
    ctx = _ctx(wl, prec="fp64")
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(ctx.num_levels)
    assert ctx.num_levels == osolve.default_levels(wl.shape) == hier.levels
    for l in range(1, ctx.num_levels):
        planes, offs = ctx.level_stencil(l)
        shape, S = ctx.level_info(l)
        assert shape == hier.shapes[l]
        assert S == (81 if wl.ndim == 3 else 21)
        A = _stencil_to_csr(planes.cpu().numpy(), offs, shape)
        ref = hier.A[l]
        err = abs(A - ref).max()
        assert err <= 1e-12 * abs(ref).max(), (l, err)


@pytest.mark.parametrize("name", ["2d_65_const", "3d_33_lin", "3d_noncubic"])
@pytest.mark.parametrize("split", [1, 4])
def test_vcycle_fp64(name, split):
    """One V-cycle (Jacobi on the finest level, GMRES relaxation below, dense coarsest)
    equals the oracle's V-cycle up to rounding, with either Galerkin-apply variant."""
    wl = CASES[name]()
    print(f"[vcycle-fp64] {name} shape={wl.shape} split={split}", flush=True)
    ctx = _ctx(wl, prec="fp64", coarse_split=split)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(ctx.num_levels)
    r = W.random_vector(wl.shape, 13)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    ref = hier.vcycle(r.ravel()).reshape(wl.shape)
    assert _rel(z, ref) <= 1e-10


@pytest.mark.parametrize("name", ["2d_65_const", "3d_33_lin"])
@pytest.mark.parametrize("split", [1, 4, 8])
def test_vcycle_mixed_close(name, split):
    """The complex-FP32 V-cycle stays within FP32 rounding of the FP64 one, with each
    Galerkin-apply variant (8: the LDS tiles over the segment-tiled planes on the 3D
    coarse levels, a partial last segment on 17^3; one lane in 2D)."""
    wl = CASES[name]()
    print(f"[vcycle-mixed] {name} shape={wl.shape} split={split}", flush=True)
    ctx = _ctx(wl, prec="mixed", coarse_split=split)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(ctx.num_levels)
    r = W.random_vector(wl.shape, 14)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    ref = hier.vcycle(r.ravel()).reshape(wl.shape)
    assert _rel(z, ref) <= 1e-4


@pytest.mark.parametrize("name", ["2d_65_const", "3d_33_lin", "3d_noncubic"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_matches_direct(name, prec):
    """Whole solve at tol 1e-10 against the oracle's direct solve: rel L2 <= 1e-6."""
    wl = CASES[name]()
    print(f"[solve] {name} shape={wl.shape} prec={prec}", flush=True)
    ctx = _ctx(wl, prec=prec)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    qh = osolve.rhs_hat(wl.rhs(), wl.tau, wl.omega)
    ref = osolve.direct_solve(p.H2up, qh).reshape(wl.shape)
    a, st = ctx.solve(_t(wl.rhs()), tol=1e-10, maxit=400)
    a = a.cpu().numpy()
    assert st["relres"] <= 1e-10
    # true residual from the oracle's matrix
    assert np.linalg.norm(p.H2up @ a.ravel() - qh.ravel()) / np.linalg.norm(qh) <= 2e-10
    assert _rel(a, ref) <= 1e-6
    u = ctx.wavefield(_t(a)).cpu().numpy()
    assert _rel(u, osolve.wavefield(a, wl.tau, wl.omega)) <= 1e-14


def test_solve_initial_guess_and_zero_rhs():
    wl = W.constant_medium(33, 2)
    print("[solve-edge] 2d 33", flush=True)
    ctx = _ctx(wl, prec="fp64")
    a, st = ctx.solve(_t(wl.rhs()), tol=1e-10, maxit=200)
    assert st["setup_ms"] > 0 and st["solve_ms"] > 0
    a2, st2 = ctx.solve(_t(wl.rhs()), tol=1e-10, maxit=200, x0=a)
    assert st2["outer_iters"] == 0 and st2["relres"] <= 1e-10
    z, st3 = ctx.solve(_t(np.zeros(wl.shape, complex)), tol=1e-10, maxit=10)
    assert np.all(z.cpu().numpy() == 0)
    _, st4 = ctx.solve(_t(wl.rhs()), tol=1e-14, maxit=3)
    from paper_1712_06091_amd import adr
    assert st4["status"] == adr.ADR_ENOCONV and st4["outer_iters"] == 3


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replays_match_eager(prec):
    """Captured V-cycles replayed several times, with unrelated eager work and
    synchronizations between replays, equal the eager V-cycle bit for bit; so do whole
    solves."""
    wl = W.linear_gradient(33, 3)
    print(f"[graph] 3d 33 prec={prec}", flush=True)
    cg = _ctx(wl, prec=prec, use_graph=1)
    ce = _ctx(wl, prec=prec, use_graph=0)
    r = torch.empty(wl.shape, dtype=torch.complex128, device="cuda")
    zg = torch.empty_like(r)
    ze = torch.empty_like(r)
    for k in range(4):
        r.copy_(_t(W.random_vector(wl.shape, 100 + k)))
        cg.vcycle(r, out=zg)
        junk = torch.randn(1000, device="cuda").cumsum(0)   # eager work between replays
        torch.cuda.synchronize()
        ce.vcycle(r, out=ze)
        torch.cuda.synchronize()
        assert torch.equal(zg, ze), f"replay {k} differs"
        del junk
    q = _t(wl.rhs())
    ag, sg = cg.solve(q, tol=1e-10, maxit=300)
    ae, se = ce.solve(q, tol=1e-10, maxit=300)
    assert sg["outer_iters"] == se["outer_iters"]
    assert torch.equal(ag, ae)


def test_full_size_3d_129_bench_configuration():
    """The benchmark workload (3D 129^3, v = 1.5 + 0.8 z) in the benchmark's launch
    configuration (mixed precision, FGMRES(5), tol 1e-6): coefficients and the FP64
    matvec match the oracle at every node, and the oracle's own H_2up confirms the true
    residual of the GPU solution."""
    wl = W.config_3d_129()
    print(f"[full-size] {wl.name} shape={wl.shape}", flush=True)
    ctx = _ctx(wl, prec="mixed")
    g, L, c = ctx.coefficients()
    og, oL, oc = ocoef.adr_coefficients(wl.tau, wl.kappa2, wl.gamma, wl.h, wl.omega, src=wl.src)
    for k in range(3):
        assert np.max(np.abs(g[k].cpu().numpy() - og[2 - k])) <= 1e-12 * np.abs(og[2 - k]).max()
    assert np.max(np.abs(L.cpu().numpy() - oL)) <= 1e-12 * np.abs(oL).max()
    H = oops.assemble_adr(og, oL, oc, wl.h, wl.omega, 0.0, src=wl.src)
    x = W.random_vector(wl.shape, 21)
    y = ctx.apply(_t(x), beta=0.0).cpu().numpy()
    scale = (abs(H) @ np.abs(x.ravel())).reshape(wl.shape)
    assert np.max(np.abs(y - (H @ x.ravel()).reshape(wl.shape)) / scale) <= 1e-13
    del x, y, scale
    a, st = ctx.solve(_t(wl.rhs()), tol=1e-6, maxit=500)
    assert st["status"] == 0 and st["relres"] <= 1e-6
    a = a.cpu().numpy().ravel()
    qh = osolve.rhs_hat(wl.rhs(), wl.tau, wl.omega).ravel()
    rel = np.linalg.norm(qh - H @ a) / np.linalg.norm(qh)
    assert rel <= 1e-6 * (1 + 1e-6), rel
    assert abs(rel - st["relres"]) <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_split_variants_agree_on_solve(prec):
    """The Galerkin-apply variants only reorder the stencil sums (the LDS tiles not even
    that): whole solves agree to rounding, and the autotuned default picks one of them.
    The LDS tiles apply to the 3D coarse levels in both precisions."""
    wl = W.linear_gradient(65, 3)
    print(f"[split-solve] shape={wl.shape} prec={prec}", flush=True)
    out = {}
    for split in (1, 4, 8, 0):
        ctx = _ctx(wl, prec=prec, coarse_split=split)
        used = [ctx.level_split(l) for l in range(1, ctx.num_levels - 1)]
        if split == 8:
            assert all(u == 8 for u in used), used
        else:
            assert all(u == split for u in used) if split else all(u in (1, 4, 8) for u in used)
        a, st = ctx.solve(_t(wl.rhs()), tol=1e-10, maxit=300)
        assert st["relres"] <= 1e-10
        out[split] = a.cpu().numpy()
        ctx.close()
    assert _rel(out[4], out[1]) <= 1e-9
    assert _rel(out[8], out[1]) <= 1e-9
    assert _rel(out[0], out[1]) <= 1e-9


TAIL_CASES = {
    # (workload, levels, tail_max_nodes): the tail starts at the first coarse level with
    # at most tail_max_nodes nodes
    "2d_129_rand_5lv": (lambda: W.random_medium(129, 2, seed=21), 5, 4225),
    "3d_33_lin_3lv": (lambda: W.linear_gradient(33, 3), 3, 5000),
}


TAIL_SKIP = ("single-workgroup coarse tail disabled: its first GPU run (2d_129_rand_5lv, tail on levels 1-3, "
             "FP64) ended in a memory aperture violation; its device code runs clean and correct on the CPU "
             "(test_tail_host.py), the launch-side cause is not found; adr_setup rejects it")


@pytest.mark.skip(reason=TAIL_SKIP)
@pytest.mark.parametrize("name", list(TAIL_CASES))
@pytest.mark.parametrize("tail", [False, True])
def test_vcycle_coarse_tail_fp64(name, tail):
    """The single-workgroup coarse tail gives the oracle's V-cycle up to rounding, like
    the multi-kernel path."""
    make, levels, tmax = TAIL_CASES[name]
    wl = make()
    print(f"[tail-fp64] {name} shape={wl.shape} tail={tail}", flush=True)
    ctx = _ctx(wl, prec="fp64", levels=levels, tail_max_nodes=tmax if tail else 0)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(levels)
    r = W.random_vector(wl.shape, 41)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    ref = hier.vcycle(r.ravel()).reshape(wl.shape)
    assert _rel(z, ref) <= 1e-10


@pytest.mark.skip(reason=TAIL_SKIP)
@pytest.mark.parametrize("name", list(TAIL_CASES))
def test_vcycle_coarse_tail_mixed_and_solves(name):
    make, levels, tmax = TAIL_CASES[name]
    wl = make()
    print(f"[tail-mixed] {name} shape={wl.shape}", flush=True)
    ctx = _ctx(wl, prec="mixed", levels=levels, tail_max_nodes=tmax)
    p = osolve.Problem(wl.kappa2, wl.tau, wl.gamma, wl.h, wl.omega, wl.src)
    hier = p.hierarchy(levels)
    r = W.random_vector(wl.shape, 42)
    z = ctx.vcycle(_t(r)).cpu().numpy()
    assert _rel(z, hier.vcycle(r.ravel()).reshape(wl.shape)) <= 1e-4
    qh = osolve.rhs_hat(wl.rhs(), wl.tau, wl.omega)
    ref = osolve.direct_solve(p.H2up, qh).reshape(wl.shape)
    a, st = ctx.solve(_t(wl.rhs()), tol=1e-10, maxit=300)
    assert st["relres"] <= 1e-10 and _rel(a.cpu().numpy(), ref) <= 1e-6
    g = W.random_vector(wl.shape, 43)
    refl = osolve.direct_solve(p.H2up.conj().T.tocsr(), osolve.rhs_hat(g, wl.tau, wl.omega)).reshape(wl.shape)
    lam, st = ctx.solve_adjoint(_t(g), tol=1e-10, maxit=300)
    assert st["relres"] <= 1e-10 and _rel(lam.cpu().numpy(), refl) <= 1e-6


def test_tuning_table_entries_steer_setup(tmp_path):
    """The autotuner writes its choice per coarse-level shape; an entry read from a table
    file replaces the timing for that shape (the previous table is restored afterwards)."""
    from paper_1712_06091_amd import adr
    wl = W.linear_gradient(65, 3)
    print("[tuning-table] 3d 65 mixed", flush=True)
    ctx = _ctx(wl, prec="mixed")
    saved = tmp_path / "saved.txt"
    adr.tuning_table_write(saved)
    rows = [l.split() for l in saved.read_text().splitlines() if not l.startswith("#")]
    shapes = {(int(r[1]), int(r[2]), int(r[3]), int(r[4])): (int(r[5]), int(r[6])) for r in rows}
    for l in range(1, ctx.num_levels - 1):
        shape, _ = ctx.level_info(l)
        assert (shape[2], shape[1], shape[0], 4) in shapes
        assert shapes[(shape[2], shape[1], shape[0], 4)][0] == ctx.level_split(l)
    ctx.close()
    forced = tmp_path / "forced.txt"
    forced.write_text("3 33 33 33 4 4 0 1.0\n")
    try:
        assert adr.tuning_table_read(forced) == 1
        c2 = _ctx(wl, prec="mixed")
        assert c2.level_split(1) == 4
        a, st = c2.solve(_t(wl.rhs()), tol=1e-10, maxit=300)
        assert st["relres"] <= 1e-10
        c2.close()
    finally:
        adr.tuning_table_read(saved)
