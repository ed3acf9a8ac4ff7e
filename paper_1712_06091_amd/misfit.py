"""Receiver misfit of point-source wavefields and its kappa^2 gradient, as a
torch.autograd.Function over the C ABI.

For sources s with travel times tau_s (held fixed), the forward pass solves
H_2up(kappa^2) a_s = q_s exp(i w tau_s) (adr_solve), forms u_s = a_s exp(-i w tau_s)
(adr_wavefield), and J = 1/2 sum_s ||R u_s - d_s||^2 (adr_receiver_residual).  The backward
pass solves H_2up^H lam_s = exp(i w tau_s) R^T r_s (adr_adjoint_source, adr_solve_adjoint)
and accumulates dJ/dkappa2 = -sum_s Re(conj(lam_s) (w^2 - i w gamma) a_s) (adr_grad_kappa2).

kappa^2 enters the operator only through the reaction term w^2 (kappa^2 - |grad tau|^2)
- i w gamma kappa^2: the travel-time derivatives are functions of tau alone (the factored
tau/|x - x0| at the source node included), so at fixed tau this gradient is complete.
"""
import torch

from . import adr


def point_source(shape, src, h, device):
    """q = e_src / h^d as a complex128 device tensor (input marshalling)."""
    q = torch.zeros(shape, dtype=torch.complex128, device=device)
    q[tuple(src)] = 1.0 / h ** len(shape)
    return q


class ReceiverMisfit(torch.autograd.Function):
    @staticmethod
    def forward(fctx, kappa2, gamma, taus, sources, h, omega, rec_idx, d_obs, options, tol, stats):
        saved = []
        J = 0.0
        for tau, src, d in zip(taus, sources, d_obs):
            c = adr.Context(kappa2.detach(), tau, gamma, h, omega, src, options=options)
            q = point_source(tau.shape, src, h, tau.device)
            a, st = c.solve(q, tol=tol, maxit=1000)
            if stats is not None:
                stats.append(("forward", st))
            if st["status"] != adr.ADR_OK:
                raise adr.AdrError(st["status"], f"forward solve did not converge: {st}")
            u = c.wavefield(a)
            r, Js = c.receiver_residual(u, rec_idx, d)
            J += Js
            saved.append((c, a, r))
        fctx.saved_solves = saved
        fctx.stats = stats
        fctx.rec_idx = rec_idx
        fctx.tol = tol
        fctx.shape = kappa2.shape
        return torch.tensor(J, dtype=torch.float64, device=kappa2.device)

    @staticmethod
    def backward(fctx, grad_out):
        grad = torch.zeros(fctx.shape, dtype=torch.float64, device=grad_out.device)
        for c, a, r in fctx.saved_solves:
            s = c.adjoint_source(fctx.rec_idx, r)
            lam, st = c.solve_adjoint(s, tol=fctx.tol, maxit=1000)
            if fctx.stats is not None:
                fctx.stats.append(("adjoint", st))
            if st["status"] != adr.ADR_OK:
                raise adr.AdrError(st["status"], f"adjoint solve did not converge: {st}")
            c.grad_kappa2(a, lam, grad)
        for c, _, _ in fctx.saved_solves:
            c.close()
        fctx.saved_solves = []
        return grad * grad_out, None, None, None, None, None, None, None, None, None, None


def receiver_misfit(kappa2, gamma, taus, sources, h, omega, rec_idx, d_obs, options=None, tol=1e-8, stats=None):
    """J(kappa^2) = 1/2 sum_s ||R u_s - d_s||^2 with a differentiable kappa^2 (float64 CUDA
    tensor).  taus: list of float64 tensors; sources: list of NumPy-order node tuples;
    rec_idx: int32 tensor of linear node indices; d_obs: list of complex128 tensors.
    ``stats``, if a list, receives ("forward" | "adjoint", solve stats) per solve."""
    if options is None:
        options = adr.default_options()
    return ReceiverMisfit.apply(kappa2, gamma, taus, sources, h, omega, rec_idx, d_obs, options, tol, stats)
