"""Differentiable rasterization as a torch.autograd.Function.

Forward: transformation, binning + sort, render forward (paper section 2.1
steps 1-2). It saves only what the backward needs: the parameters, the
projected records and the sorted instance lists (the Z-buffer, which the
paper notes is used in both forward and backward, appendix A.2), and per
pixel the final transmittance and the last-contributor position. Backward
recomputes the blend in reverse (gs_render_bwd) - no per-pixel history is
stored. Works in float32 and float64 (for finite-difference checks).
"""
from __future__ import annotations

import torch

from . import _lib
from . import raster as R


class GaussianRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, cams: R.Cameras, bg=(0.0, 0.0, 0.0), sched: R.Sched | None = None,
                headroom: float = 1.25):
        P = params.detach().contiguous()
        n = P.shape[1]
        proj = R.gs_project(P, cams)
        tiles, _ = R.projected_side_arrays(proj)
        K = int(tiles.sum(dtype=torch.int64).item())
        bins = R.Bins(n, cams, max(int(K * headroom), 16))
        R.gs_bin_sort(proj, n, cams, bins, check_capacity=True)
        rgb, T, last = R.gs_render_fwd(proj, n, bins, cams, bg, sched)
        ctx.save_for_backward(P, proj, T, last)
        ctx.bins, ctx.cams, ctx.bg, ctx.sched = bins, cams, bg, sched
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb: torch.Tensor):
        P, proj, T, last = ctx.saved_tensors
        grad = torch.zeros_like(P)
        dproj = torch.zeros(ctx.cams.n, P.shape[1], _lib.GS_REC, dtype=P.dtype, device=P.device)
        R.gs_render_bwd(P, proj, ctx.bins, ctx.cams, T, last, grad_rgb.contiguous(), grad, ctx.bg, ctx.sched,
                        dprojected=dproj)
        return grad, None, None, None, None


def rasterize(params: torch.Tensor, cams: R.Cameras, bg=(0.0, 0.0, 0.0), sched: R.Sched | None = None):
    """Images of all views, concatenated planar [3][H][W] per view (flat)."""
    return GaussianRasterize.apply(params, cams, bg, sched)
