"""The treecode energy as a differentiable torch function.

Forward builds an octree from the given positions and charges and evaluates
the treecode energy of Sec. 3; it keeps nothing of the tree.  Backward builds
the tree again from the saved positions and charges (every moment recomputed,
none stored between the passes) and evaluates the exact gradient of that same
energy for the interaction lists its traversal makes (dE/dr per ion, and
dE/dq).  All the work runs in the HIP library; this module marshals tensors.
"""
from __future__ import annotations

import torch

from . import bhmc


class TreecodeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, z, q, params):
        tree = bhmc.Tree(params, x.detach(), y.detach(), z.detach(), q.detach(), device=x.device)
        try:
            E = tree.energy()
        finally:
            tree.close()
        ctx.params = dict(params)
        ctx.save_for_backward(x.detach(), y.detach(), z.detach(), q.detach())
        return torch.tensor(E, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, grad_out):
        x, y, z, q = ctx.saved_tensors
        tree = bhmc.Tree(ctx.params, x, y, z, q, device=x.device)
        try:
            _, g, gq = tree.energy_grad()
        finally:
            tree.close()
        return grad_out * g[:, 0], grad_out * g[:, 1], grad_out * g[:, 2], grad_out * gq, None


def treecode_energy(x, y, z, q, params) -> torch.Tensor:
    """E(x, y, z, q) of the treecode (float64 device tensors of n ions)."""
    return TreecodeEnergy.apply(x, y, z, q, params)
