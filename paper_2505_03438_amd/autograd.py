"""Differentiable Lennard-Jones forces: a torch.autograd.Function over the
C-ABI calls md_compute_forces (forward) and md_forces_backward (the adjoint
kernel).  Marshalling only; both passes run in the HIP library.

For a loss L(F) of the forces F(x; theta), the backward pass returns
dL/dx (FP64, the positions' dtype) and dL/dtheta for the per-type parameters
theta = (eps_0 .. eps_{T-1}, sig_0 .. sig_{T-1}), with pair parameters mixed
by the Lorentz-Berthelot rules (Sec. 2.1; the mixing's chain rule is applied
in the library).  The cutoffs are fixed by the handle's configuration and
are not differentiated.
"""
from __future__ import annotations

import torch

from . import mdlj as M


class LJForces(torch.autograd.Function):
    """forces = LJForces.apply(pos, lj, handle, type).

    pos: (3, n) float64 device tensor in the cell order of the handle's last
    md_build_cells (the cells, and lists if any, must be valid for pos);
    lj: (2 T,) float64 device tensor; type: (n,) int32 device tensor.
    Returns the (3, n) forces in the handle's precision (float32 or float64).
    """

    @staticmethod
    def forward(ctx, pos, lj, handle, type):
        pos_c = pos.detach().contiguous()
        lj_c = lj.detach().contiguous()
        force = torch.empty((3, handle.n), dtype=handle.real, device=pos.device)
        M.md_compute_forces(handle, pos_c, type, lj_c, force)
        ctx.handle = handle
        ctx.save_for_backward(pos_c, lj_c, type)
        return force

    @staticmethod
    def backward(ctx, grad_force):
        pos, lj, type = ctx.saved_tensors
        h = ctx.handle
        g = grad_force.to(h.real).contiguous()
        grad_pos = torch.zeros((3, h.n), dtype=torch.float64, device=pos.device)
        grad_lj = torch.zeros(lj.numel(), dtype=torch.float64, device=pos.device)
        M.md_forces_backward(h, pos, type, lj, g, grad_pos, grad_lj)
        return (grad_pos if ctx.needs_input_grad[0] else None,
                grad_lj if ctx.needs_input_grad[1] else None, None, None)


def lj_forces(handle, pos, type, lj):
    """Functional form of LJForces."""
    return LJForces.apply(pos, lj, handle, type)
