"""Autograd form: the coupled CP reconstruction loss
F = sum_s 1/2 ||M^(s) - [[lambda^(s); U^(1,s), U^(2,s), U^(3,s)]]||_F^2 as a
torch.autograd.Function.  One library call evaluates F and every partial
gradient (the same gradient the APG steps use: eq. solbpgU / solbpgG); the
backward pass scales the saved gradients by the incoming one.  Shared columns
are tied by the caller (e.g. U^(n,s) = cat(U_C, U_I^(s))), so autograd sums
their per-block gradients.
"""
from __future__ import annotations

import torch


class CoupledCPLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, *params):
        S = model.S
        U = [[params[n * S + s] for s in range(S)] for n in range(3)]
        lam = list(params[3 * S:])
        F, gU, glam = model.loss_grad([[u.detach() for u in per] for per in U], [l.detach() for l in lam], coupled=False)
        ctx.save_for_backward(*[gU[n][s] for n in range(3) for s in range(S)], *glam)
        return torch.tensor(F, dtype=torch.float64, device=params[0].device)

    @staticmethod
    def backward(ctx, gout):
        return (None, *[g * gout.to(g.dtype) for g in ctx.saved_tensors])


def coupled_cp_loss(model, U, lam):
    """F at (U [n][s], lam [s]); differentiable with respect to every tensor."""
    S = model.S
    return CoupledCPLoss.apply(model, *[U[n][s] for n in range(3) for s in range(S)], *lam)
