"""torch.autograd wrappers of the HIP solve and its hand-written adjoint.

MacroHDGSolve(kappa, beta) -> U  runs factor_local + solve + recover_local;
its backward calls mhdg_adjoint (transposed GMRES on S^T and A_K^-T solves
with the stored LU factors) and returns dJ/dkappa (per macro) and dJ/dbeta.
MassApply(v) -> M v (macro mass matrices, self-adjoint) lets objectives such
as J = ||u_h - u_obs||^2_{L2} be written in torch.  Both are marshalling only:
every step runs in the library.
"""
from __future__ import annotations

import torch

from . import mhdg


def _forward(mesh, kappa, beta, f, g, rtol, restart, folded):
    s = mesh.sizes
    dev = kappa.device
    mesh.factor_local(kappa.detach(), (float(beta[0]), float(beta[1])), 1.0)
    if folded:
        mesh.fold_operator()
    lam = torch.zeros(s.n_trace, dtype=torch.float64, device=dev)
    mesh.solve(f, g, lam, rtol=rtol, restart=restart, max_iter=max(50000, 2 * restart),
               folded=folded)
    qu = torch.empty(s.n_local, dtype=torch.float64, device=dev)
    mesh.recover_local(lam, qu)
    return lam, qu


class MacroHDGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, beta, mesh, f, g, rtol, restart, folded):
        beta_h = beta.detach().cpu()
        lam, qu = _forward(mesh, kappa, beta_h, f, g, rtol, restart, folded)
        ctx.mesh, ctx.f, ctx.g, ctx.rtol, ctx.restart = mesh, f, g, rtol, restart
        ctx.folded = folded
        # the handle's state counter after this forward: any later call that
        # changes its factors or stored right-hand side moves it on
        ctx.gen = mesh.state_gen
        ctx.save_for_backward(kappa.detach().clone(), beta_h.clone(), lam, qu)
        return qu

    @staticmethod
    def backward(ctx, grad_qu):
        kappa, beta_h, lam, qu = ctx.saved_tensors
        mesh = ctx.mesh
        ctx.reforwarded = mesh.state_gen != ctx.gen
        if ctx.reforwarded:
            # another solve ran since: restore this problem's factors and traces
            lam, qu = _forward(mesh, kappa, beta_h, ctx.f, ctx.g, ctx.rtol, ctx.restart,
                               ctx.folded)
        s = mesh.sizes
        dev = kappa.device
        dk = torch.empty(s.n_macro, dtype=torch.float64, device=dev)
        db = torch.empty(2, dtype=torch.float64, device=dev)
        psi_lam = torch.empty(max(s.n_trace, 1), dtype=torch.float64, device=dev)
        psi_U = torch.empty(s.n_local, dtype=torch.float64, device=dev)
        mesh.adjoint(lam, qu, grad_qu.contiguous(), psi_lam, psi_U, dk, db, rtol=ctx.rtol,
                     restart=ctx.restart, folded=ctx.folded)
        mesh.last_backward_reforwarded = ctx.reforwarded
        return dk, db.to(beta_h.device if beta_h.device.type == "cuda" else "cpu"), None, None, \
            None, None, None, None


def solve(kappa, beta, mesh, f, g, rtol=1e-12, restart=300, folded=False):
    """Differentiable U(kappa, beta) (local vectors [q_x | q_y | u] per macro).
    folded=True runs both GMRES solves on the folded macro operators."""
    return MacroHDGSolve.apply(kappa, beta, mesh, f, g, rtol, restart, folded)


class MassApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, mesh):
        out = torch.empty_like(v)
        mesh.mass_apply(v.contiguous(), out)
        ctx.mesh = mesh
        return out

    @staticmethod
    def backward(ctx, grad):
        out = torch.empty_like(grad)
        ctx.mesh.mass_apply(grad.contiguous(), out)
        return out, None


def l2_misfit(mesh, qu, u_obs_qu):
    """J = ||u_h - u_obs||^2_{L2(Omega)} over the u field (local vectors)."""
    s = mesh.sizes
    Q = s.n_nodes // s.n_macro
    d = qu - u_obs_qu
    mask = torch.zeros(s.n_macro, 3, Q, dtype=torch.float64, device=qu.device)
    mask[:, 2, :] = 1.0
    d = d * mask.reshape(-1)
    return torch.dot(d, MassApply.apply(d, mesh))
