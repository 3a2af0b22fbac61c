"""The MLS dispersion energy as a differentiable PyTorch function.

``MLSDispersion.apply(pos, c6, plan) -> E`` runs one evaluation through the
C ABI (``mls_evaluate``) with forces and dE/dC6 requested and keeps them for
the backward pass, which is hand-written: dE/dpos = -F and dE/dC6 come
straight from the library (F = -grad E of the MLS energy; dE/dC6_i from the
per-atom potential, Sec. II.B with xi_i = sqrt(C6_i)).  No second launch;
double backward is not supported.
"""
from __future__ import annotations

import torch

__all__ = ["MLSDispersion", "mls_energy"]


class MLSDispersion(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, c6, plan):
        res = plan.evaluate(pos.detach().contiguous(), c6.detach().contiguous(), forces=True, dE_dc6=True)
        ctx.save_for_backward(res.forces, res.dE_dc6)
        return res.energy.reshape(())

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_e):
        forces, de_dc6 = ctx.saved_tensors
        g_pos = -grad_e * forces if ctx.needs_input_grad[0] else None
        g_c6 = grad_e * de_dc6 if ctx.needs_input_grad[1] else None
        return g_pos, g_c6, None


def mls_energy(pos, c6, plan):
    """Differentiable MLS energy (a 0-d float64 tensor on the plan's device)."""
    return MLSDispersion.apply(pos, c6, plan)
