"""GPU batched shots: lockstep solves over several streams equal individual solves."""
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
    for i, w in enumerate(wls):
        c = adr.Context(shots[i]["kappa2"], shots[i]["tau"], shots[i]["gamma"], w.h, w.omega, w.src, options=opts)
        a, s1 = c.solve(qs[i], tol=1e-8, maxit=400)
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
