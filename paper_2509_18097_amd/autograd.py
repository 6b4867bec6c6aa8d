"""torch.autograd functions with hand-written adjoints (libpdg kernels).

``DeformFn``   warp x + level_scale * sum_l trilerp(G_l, x) (paper Eq. 1);
               backward gives dL/dG (the transpose of the interpolation,
               deterministic) and dL/dx (identity plus the position Jacobian).
``ChamferFn``  the two directional terms of the robust Chamfer distance
               (Eq. 11-13) as a float64 (2,) tensor plus the nearest-neighbour
               indices; backward gives dL/da from the saved indices (the
               Gaussian weight is differentiated, b is data).

Forward and backward both run in the library; torch provides tensors and the
current stream only.
"""
from __future__ import annotations

import torch

from . import _lib as L


class DeformFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grids, x, res, level_scale=None):
        ctx.res = tuple(res)
        ctx.level_scale = level_scale
        ctx.save_for_backward(grids, x)
        return L.deform(grids.contiguous(), x.contiguous(), res, level_scale)

    @staticmethod
    def backward(ctx, gout):
        grids, x = ctx.saved_tensors
        gg, gx = L.deform_backward(grids.contiguous(), x.contiguous(), gout.contiguous(), ctx.res,
                                   ctx.level_scale, need_grids=ctx.needs_input_grad[0],
                                   need_x=ctx.needs_input_grad[1])
        return gg, gx, None, None


class ChamferFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b, alpha=5.56, mode="fp32"):
        a = a.contiguous()
        b = b.contiguous()
        loss, nn_a, nn_b, _ = L.chamfer(a, b, alpha=alpha, mode=mode)
        ctx.alpha = float(alpha)
        ctx.save_for_backward(a, b, nn_a, nn_b)
        ctx.mark_non_differentiable(nn_a, nn_b)
        return loss, nn_a, nn_b

    @staticmethod
    def backward(ctx, gloss, _gna, _gnb):
        a, b, nn_a, nn_b = ctx.saved_tensors
        if not ctx.needs_input_grad[0]:
            return None, None, None, None
        w = gloss.detach().to(torch.float64).contiguous()
        ga = L.chamfer_backward(a, b, nn_a, nn_b, w, alpha=ctx.alpha)
        return ga, None, None, None


def deform(grids, x, res, level_scale=None):
    return DeformFn.apply(grids, x, res, level_scale)


def chamfer(a, b, alpha=5.56, mode="fp32"):
    """(loss (2,) float64 per direction, nn_a, nn_b); CD_R = loss.sum()."""
    return ChamferFn.apply(a, b, alpha, mode)
