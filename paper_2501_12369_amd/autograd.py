"""``torch.autograd.Function`` over the libdarb C ABI.

The forward renders through preprocess -> bin/sort -> raster forward and keeps
only per-splat projected records, the sorted instance list and the per-pixel
checkpoint (final transmittance, position of the last blended instance); the
backward recomputes every per-pair quantity from them (darb_raster_bwd) and
chains through the projection (darb_preprocess_bwd).  Parameters are
structure-of-arrays tensors on the GPU: means/scales [3, n], quats [4, n]
(w, x, y, z), opacity [n], sh [(deg+1)^2, 3, n].
"""
from __future__ import annotations

import torch

from . import pipeline


class DarbRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacity, sh, cam: dict, kernel, opts: dict | None, sh_degree: int):
        splats = dict(means=means.detach().contiguous(), scales=scales.detach().contiguous(),
                      quats=quats.detach().contiguous(), opacity=opacity.detach().contiguous(),
                      sh=sh.detach().contiguous(), sh_degree=int(sh_degree))
        frame = pipeline.render(splats, cam, kernel, opts)
        ctx.frame = frame
        ctx.splats = splats
        ctx.cam = cam
        ctx.kernel = kernel
        ctx.opts = opts
        return frame.image.clone()

    @staticmethod
    def backward(ctx, grad_image):
        g2d, g3d = pipeline.render_backward(ctx.frame, grad_image.contiguous(), ctx.splats, ctx.cam, ctx.kernel,
                                            ctx.opts)
        ctx.frame = None
        return g3d["means"], g3d["scales"], g3d["quats"], g3d["opacity"], g3d["sh"], None, None, None, None


def rasterize(means, scales, quats, opacity, sh, cam: dict, kernel="half_cos", opts: dict | None = None,
              sh_degree: int | None = None):
    """Differentiable render of one view; returns the [3, H, W] image."""
    if isinstance(kernel, str):
        kernel = pipeline.KERNELS[kernel]
    if sh_degree is None:
        sh_degree = int(round(sh.shape[0] ** 0.5)) - 1
    return DarbRasterize.apply(means, scales, quats, opacity, sh, cam, kernel, opts, sh_degree)
