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
    def forward(ctx, means, scales, quats, opacity, sh, cam: dict, kernel, opts: dict | None, sh_degree: int,
                owner=None, keep: bool = True):
        splats = dict(means=means.detach().contiguous(), scales=scales.detach().contiguous(),
                      quats=quats.detach().contiguous(), opacity=opacity.detach().contiguous(),
                      sh=sh.detach().contiguous(), sh_degree=int(sh_degree))
        frame = owner.render(splats, cam) if owner is not None else pipeline.render(splats, cam, kernel, opts)
        image = frame.image.clone()
        if owner is not None and not (keep and any(ctx.needs_input_grad[:5])):
            owner.release(frame)  # no backward will read this checkpoint
            frame = None
        ctx.owner = owner
        ctx.frame = frame
        ctx.splats = splats
        ctx.cam = cam
        ctx.kernel = kernel
        ctx.opts = opts
        return image

    @staticmethod
    def backward(ctx, grad_image):
        if ctx.frame is None:
            raise RuntimeError("DarbRasterize: backward called twice on one forward")
        grads = None
        zeroed = False
        if ctx.owner is not None:  # reuse the owner's 2D-gradient buffers; fresh 3D gradients (returned)
            n, deg = ctx.frame.n, ctx.splats["sh_degree"]
            grads = (ctx.owner.grads2d(n), pipeline.alloc_grads(n, deg, "cuda")[1])
            zeroed = ctx.owner.take_cleared_grads2d(ctx.frame)
        g2d, g3d = pipeline.render_backward(ctx.frame, grad_image.contiguous(), ctx.splats, ctx.cam, ctx.kernel,
                                            ctx.opts, grads=grads, g2d_zeroed=zeroed)
        if ctx.owner is not None:
            ctx.owner.release(ctx.frame)
        ctx.frame = None
        return (g3d["means"], g3d["scales"], g3d["quats"], g3d["opacity"], g3d["sh"], None, None, None, None, None,
                None)


def rasterize(means, scales, quats, opacity, sh, cam: dict, kernel="half_cos", opts: dict | None = None,
              sh_degree: int | None = None):
    """Differentiable render of one view; returns the [3, H, W] image."""
    if isinstance(kernel, str):
        kernel = pipeline.KERNELS[kernel]
    if sh_degree is None:
        sh_degree = int(round(sh.shape[0] ** 0.5)) - 1
    return DarbRasterize.apply(means, scales, quats, opacity, sh, cam, kernel, opts, sh_degree)


class Rasterizer:
    """Differentiable renderer that keeps its device buffers between steps: no
    allocation per step, and the instance count is read back only to check for
    a capacity overflow (then the list grows by ``k_margin`` and the view is
    rendered again).  The forward runs the preprocess's colour part on a second
    stream beside the binning and clears the backward's 2D-gradient buffers in
    its raster kernel; the next backward then skips its own clearing (only the
    backward of the latest forward, and only once: any other backward finds
    the buffers used and clears them itself).

    Each forward holds its own frame (projected records, sorted list,
    checkpoint) until its backward has run, so several forwards may precede
    their backwards (a loss summed over views rendered one after another);
    frames return to a pool keyed by (n, W, H) and are reused by later
    forwards."""

    def __init__(self, kernel="half_cos", opts: dict | None = None, k_margin: float = 1.1):
        self.kernel = pipeline.KERNELS[kernel] if isinstance(kernel, str) else kernel
        self.opts = opts
        self.k_margin = k_margin
        self._pool = {}
        self._grads = None
        self._cleared_by = None  # the frame whose forward cleared the 2D-gradient buffers
        self._side = None

    def render(self, splats: dict, cam: dict):
        n, W, H = int(splats["means"].shape[1]), int(cam["width"]), int(cam["height"])
        g2 = self.grads2d(n)
        free = self._pool.get((n, W, H))
        if not free:
            fr = pipeline.render(splats, cam, self.kernel, self.opts, k_capacity=max(4 * n, 1 << 16), zero_g2d=g2)
            self._cleared_by = fr
            return fr
        fr = free.pop()
        if self._side is None:
            self._side = torch.cuda.Stream()
        pipeline.forward_overlapped(splats, cam, self.kernel, fr, self._side, self.opts, zero_g2d=g2)
        if int(fr.overflow[0].item()) != 0:  # too many instances: grow and render again
            K = int(fr.k_dev[0].item())
            pipeline._grow(fr, int(K * self.k_margin), fr.vals.device)
            pipeline.render(splats, cam, self.kernel, self.opts, frame=fr, read_k=True, zero_g2d=g2)
        self._cleared_by = fr
        return fr

    def release(self, frame) -> None:
        """Return a frame whose checkpoint is no longer needed to the pool."""
        self._pool.setdefault((frame.n, frame.width, frame.height), []).append(frame)

    def grads2d(self, n: int):
        if self._grads is None or self._grads["opacity"].numel() != n:
            self._grads = pipeline.alloc_grads(n, 0, "cuda")[0]
            self._cleared_by = None
        return self._grads

    def take_cleared_grads2d(self, frame) -> bool:
        """True when ``frame``'s forward was the last to clear the 2D-gradient
        buffers and no backward has used them since (then they are zero)."""
        c = self._cleared_by is frame
        self._cleared_by = None
        return c

    def __call__(self, means, scales, quats, opacity, sh, cam: dict, sh_degree: int | None = None):
        if sh_degree is None:
            sh_degree = int(round(sh.shape[0] ** 0.5)) - 1
        # a forward under no_grad keeps no checkpoint (grad mode is off inside forward itself)
        keep = torch.is_grad_enabled()
        return DarbRasterize.apply(means, scales, quats, opacity, sh, cam, self.kernel, self.opts, sh_degree, self,
                                   keep)
