"""GPU batched shots: shot groups (one launch per phase for all problems of a grid
shape) give, per problem, the single solve with full restart cycles bit for bit."""
import numpy as np
import pytest

from oracle import solve as osolve
from paper_1712_06091_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _shot(wl):
    return {"kappa2": _t(wl.kappa2, torch.float64), "tau": _t(wl.tau, torch.float64),
            "gamma": _t(wl.gamma, torch.float64), "h": wl.h, "omega": wl.omega, "src": wl.src}


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batch_matches_individual_solves(prec):
    from paper_1712_06091_amd import adr
    wls = W.batch_2d(count=6, seed=7, sizes=(65, 129)) + [W.linear_gradient(33, 3), W.random_medium(33, 3, seed=8)]
    print(f"[batch] {len(wls)} shots prec={prec} sizes={[w.shape for w in wls]}", flush=True)
    opts = adr.default_options(prec=prec)
    shots = [_shot(w) for w in wls]
    qs = [_t(w.rhs(), torch.complex128) for w in wls]
    outs = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in wls]
    b = adr.Batch(shots, options=opts, nstreams=3)
    st, stats = b.solve(qs, outs, tol=1e-8, maxit=400)
    assert st == adr.ADR_OK
    single = adr.default_options(prec=prec, full_cycles=1)
    for i, w in enumerate(wls):
        c = adr.Context(shots[i]["kappa2"], shots[i]["tau"], shots[i]["gamma"], w.h, w.omega, w.src, options=single)
        a, s1 = c.solve(qs[i], tol=1e-8, maxit=400)
        assert s1["outer_iters"] % 5 == 0 or s1["outer_iters"] >= 400, i
        assert s1["outer_iters"] == stats[i]["outer_iters"], i
        assert torch.equal(a, outs[i]), i
        c.close()
    # two shots against the oracle's direct solve
    for i in (0, 6):
        w = wls[i]
        p = osolve.Problem(w.kappa2, w.tau, w.gamma, w.h, w.omega, w.src)
        ref = osolve.direct_solve(p.H2up, osolve.rhs_hat(w.rhs(), w.tau, w.omega))
        got = outs[i].cpu().numpy().ravel()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-6
    b.close()


def test_batch_repeated_solves_and_masking():
    """Two batch solves in a row with different right-hand sides (the device flags are
    re-armed), shots of one group converging at different iterations, and a zero
    right-hand side (finished at START) inside a group."""
    from paper_1712_06091_amd import adr
    wls = [W.random_medium(65, 2, seed=s) for s in (31, 32, 33)] + [W.constant_medium(65, 2)]
    print(f"[batch-repeat] {len(wls)} shots", flush=True)
    opts = adr.default_options(prec="mixed")
    shots = [_shot(w) for w in wls]
    b = adr.Batch(shots, options=opts, nstreams=2)
    single = adr.default_options(prec="mixed", full_cycles=1)
    ctxs = [adr.Context(sh["kappa2"], sh["tau"], sh["gamma"], w.h, w.omega, w.src, options=single)
            for sh, w in zip(shots, wls)]
    for rnd in range(2):
        qs = [_t(W.random_vector(w.shape, 100 * rnd + i), torch.complex128) for i, w in enumerate(wls)]
        if rnd == 1:
            qs[2] = torch.zeros_like(qs[2])
        outs = [torch.full(w.shape, 7.0 + 0j, dtype=torch.complex128, device="cuda") for w in wls]
        st, stats = b.solve(qs, outs, tol=1e-9, maxit=300)
        assert st == adr.ADR_OK
        for i in range(len(wls)):
            a, s1 = ctxs[i].solve(qs[i], tol=1e-9, maxit=300)
            assert s1["outer_iters"] == stats[i]["outer_iters"], (rnd, i)
            assert torch.equal(a, outs[i]), (rnd, i)
        if rnd == 1:
            assert stats[2]["outer_iters"] == 0 and torch.count_nonzero(outs[2]) == 0
    for c in ctxs:
        c.close()
    b.close()


@pytest.mark.parametrize("variant", ["kcycle", "central", "h1up", "shift"])
def test_batch_option_variants(variant):
    """The per-problem operator parameters of a shot group (advection scheme, the blend of
    the solved operator, the shift, the cycle) reach every problem: each equals its single
    solve with full restart cycles bit for bit."""
    from paper_1712_06091_amd import adr
    kw = {"kcycle": dict(cycle="k"), "central": dict(advection="central", beta=0.0),
          "h1up": dict(beta=1.0, outer_beta=1.0, cycle="k"), "shift": dict(shift_alpha=0.3)}[variant]
    wls = [W.random_medium(65, 2, seed=s) for s in (41, 42)] + [W.constant_medium(65, 2)]
    print(f"[batch-variant] {variant} shots={len(wls)} omegas={[round(w.omega, 2) for w in wls]}", flush=True)
    shots = [_shot(w) for w in wls]
    qs = [_t(w.rhs(), torch.complex128) for w in wls]
    outs = [torch.empty(w.shape, dtype=torch.complex128, device="cuda") for w in wls]
    b = adr.Batch(shots, options=adr.default_options(prec="mixed", **kw), nstreams=2)
    st, stats = b.solve(qs, outs, tol=1e-8, maxit=400)
    assert st == adr.ADR_OK
    single = adr.default_options(prec="mixed", full_cycles=1, **kw)
    for i, w in enumerate(wls):
        c = adr.Context(shots[i]["kappa2"], shots[i]["tau"], shots[i]["gamma"], w.h, w.omega, w.src, options=single)
        a, s1 = c.solve(qs[i], tol=1e-8, maxit=400)
        assert s1["outer_iters"] == stats[i]["outer_iters"], i
        assert torch.equal(a, outs[i]), i
        c.close()
    b.close()
