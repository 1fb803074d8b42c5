"""EOFA action as a torch.autograd.Function (eqs. (2.5) and (3.2)).

forward:  S(U) = phi^dag M_EOFA(U) phi, through eofa_solve (two Cayley-form
          CG solves on the GPU).
backward: dS/dU from the hand-written adjoint kernel (eofa_force), which
          forms the outer products of the saved solutions chi_L, chi_R.
The gradient follows torch's convention for a real function of complex
input: dS = Re sum tr(G^dag dU).  No gradient flows to phi.
"""
from __future__ import annotations

import torch

from .api import Context


class EOFAAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, phi, eofa_ctx: Context, m1: float, m2: float, solver: dict):
        eofa_ctx.update_gauge(U.detach().contiguous())
        chiL, chiR, _, S, _ = eofa_ctx.eofa_solve(phi, m1, m2, want_mphi=False, **solver)
        ctx.save_for_backward(chiL, chiR)
        ctx.eofa = (eofa_ctx, m1, m2, solver)
        return torch.tensor(S, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, grad_S):
        chiL, chiR = ctx.saved_tensors
        eofa_ctx, m1, m2, solver = ctx.eofa
        _, G, _ = eofa_ctx.eofa_force(m1, m2, chiL=chiL, chiR=chiR, want_grad=True)
        return grad_S * G, None, None, None, None, None


def eofa_action(U, phi, eofa_ctx: Context, m1: float, m2: float, **solver):
    """S = phi^dag M_EOFA phi with autograd support in U."""
    return EOFAAction.apply(U, phi, eofa_ctx, float(m1), float(m2), solver)
