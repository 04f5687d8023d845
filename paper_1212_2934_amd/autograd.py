"""torch.autograd wrapper of the Barnes-Hut field and energy.

BHEnergy.apply(pos, mom, hext, handle) -> (H, E) runs bh_build + bh_field; its backward runs
bh_field_backward, the adjoint traversal, with the tree of the forward positions (the structure is held
fixed, as the derivative of the piecewise-constant tree is zero almost everywhere).  Tensors are (3, n) or
(B, 3, n) float64 CUDA tensors; hext is (3,) or (B, 3).
"""
from __future__ import annotations

import torch

from .binding import BarnesHut


class BHEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, mom, hext, handle: BarnesHut):
        pos, mom = pos.contiguous(), mom.contiguous()
        hext = hext.contiguous()
        handle.build(pos)
        H, E = handle.field(mom, hext)
        ctx.save_for_backward(pos, mom, hext)
        ctx.handle = handle
        ctx.hext_shape = hext.shape
        return H, E

    @staticmethod
    def backward(ctx, gH, gE):
        pos, mom, hext = ctx.saved_tensors
        h = ctx.handle
        h.build(pos)  # the handle may have been used for other positions since the forward
        gH = None if gH is None else gH.contiguous()
        gE = None if gE is None else gE.reshape(h.batch).contiguous()
        dpos, dmom, dhext = h.field_backward(mom, hext, gH=gH, gE=gE, want_dhext=True)
        return dpos, dmom, dhext.reshape(ctx.hext_shape), None


def bh_energy(pos, mom, hext, handle: BarnesHut):
    """(H, E) with gradients flowing to pos, mom and hext through the adjoint traversal."""
    return BHEnergy.apply(pos, mom, hext, handle)
