"""torch.autograd binding of the renderer: forward = plx_render_fwd, backward
= plx_render_bwd (reverse replay with recomputed transmittance; only the rays,
the per-ray optical depth and the batch's segment lists are saved)."""
from __future__ import annotations

import torch

from . import binding as B


class RenderFn(torch.autograd.Function):
    """rgb = RenderFn.apply(params, grid, rays_o, rays_d, bg).

    ``params`` is the grid's FP32 record tensor [M, 32] (``grid.data`` for
    FP32 grids, ``grid.master`` for 16-bit ones); its gradient has the same
    record layout (slots 0..26 SH, slot 28 density).  The forward reads the
    grid's stored records."""

    @staticmethod
    def forward(ctx, params, grid, rays_o, rays_d, bg):
        n = rays_o.shape[0]
        rgb = torch.empty(n, 3, dtype=torch.float32, device=rays_o.device)
        tau = torch.empty(n, dtype=torch.float32, device=rays_o.device)
        desc = grid.desc()
        bins = B.make_bins(desc, rays_o, rays_d)
        B.plx_render_fwd(desc, rays_o, rays_d, rgb, tau, bg, bins=bins)
        ctx.save_for_backward(rays_o, rays_d, tau)
        ctx.grid = grid
        ctx.bins = bins
        ctx.bg = tuple(bg)
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        rays_o, rays_d, tau = ctx.saved_tensors
        g = ctx.grid
        grad = torch.zeros(g.n_vox, B.REC_SLOTS, dtype=torch.float32, device=rays_o.device)
        touched = torch.zeros(g.n_vox, dtype=torch.uint8, device=rays_o.device)
        B.plx_render_bwd(g.desc(), rays_o, rays_d, grad_rgb.contiguous().float(), tau, grad,
                         touched, ctx.bg, bins=ctx.bins)
        return grad, None, None, None, None


def render(grid, rays_o, rays_d, bg=(1.0, 1.0, 1.0)) -> torch.Tensor:
    """Differentiable render of a ray batch with respect to the grid's FP32
    records (set ``grid.param_records().requires_grad_()`` first)."""
    return RenderFn.apply(grid.param_records(), grid, rays_o, rays_d, tuple(bg))
