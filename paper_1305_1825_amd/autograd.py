"""The treecode energy as a differentiable torch function.

Forward builds an octree from the given positions and charges (so every
moment is computed fresh from them), evaluates the treecode energy of Sec. 3
and, in the same library call, its exact gradient for the interaction lists
the traversal makes (dE/dr per ion, and dE/dq).  Backward only scales that
gradient.  All the work runs in the HIP library; this module marshals tensors.
"""
from __future__ import annotations

import torch

from . import bhmc


class TreecodeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, z, q, params):
        tree = bhmc.Tree(params, x.detach(), y.detach(), z.detach(), q.detach(), device=x.device)
        try:
            E, g, gq = tree.energy_grad()
        finally:
            tree.close()
        ctx.save_for_backward(g, gq)
        return torch.tensor(E, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, grad_out):
        g, gq = ctx.saved_tensors
        return grad_out * g[:, 0], grad_out * g[:, 1], grad_out * g[:, 2], grad_out * gq, None


def treecode_energy(x, y, z, q, params) -> torch.Tensor:
    """E(x, y, z, q) of the treecode (float64 device tensors of n ions)."""
    return TreecodeEnergy.apply(x, y, z, q, params)
