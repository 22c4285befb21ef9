"""Differentiable interpolate / spread pair.

Interpolation U = I(X) u and spreading f = I(X)^T F share the weights
w_kn = phi(r_x) phi(r_y) phi(r_z) (Sec. 2.2), so each is the other's adjoint:
the backward of interpolate with respect to the leaf field is spread of the
upstream gradient, and the backward of spread with respect to the forces is
interpolate.  Gradients with respect to the point positions go through the
derivative of phi, the host leaf held fixed.  Each backward is one pass over
the points that computes both gradients (ot_interp_backward,
ot_spread_backward).
"""
from __future__ import annotations

import torch


class InterpolateFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, field, pos, tree, mode):
        ctx.tree, ctx.mode = tree, mode
        ctx.save_for_backward(field, pos)
        return tree.interpolate(field, pos)

    @staticmethod
    def backward(ctx, g):
        field, pos = ctx.saved_tensors
        need_f, need_x = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_f or need_x):
            return None, None, None, None
        gf, gx = ctx.tree.interp_backward(field, g.contiguous(), pos, mode=ctx.mode, need_field=need_f,
                                          need_pos=need_x)
        return gf, gx, None, None


class SpreadFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, force, pos, tree, mode):
        ctx.tree = tree
        ctx.save_for_backward(force, pos)
        return tree.spread(force, pos, mode=mode)

    @staticmethod
    def backward(ctx, g):
        force, pos = ctx.saved_tensors
        need_F, need_x = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_F or need_x):
            return None, None, None, None
        gF, gx = ctx.tree.spread_backward(g.contiguous(), force, pos, need_force=need_F, need_pos=need_x)
        return gF, gx, None, None


def interpolate(tree, field: torch.Tensor, pos: torch.Tensor, mode: str = "atomic") -> torch.Tensor:
    """Differentiable interpolation; `mode` is the spreading mode of its backward."""
    return InterpolateFn.apply(field, pos, tree, mode)


def spread(tree, force: torch.Tensor, pos: torch.Tensor, mode: str = "atomic") -> torch.Tensor:
    return SpreadFn.apply(force, pos, tree, mode)
