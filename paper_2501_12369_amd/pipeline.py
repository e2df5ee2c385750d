"""Device buffers and the call sequence of one render (forward and backward).

Torch only allocates device memory and supplies the stream; every stage runs
in libdarb through :mod:`native`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from . import native

# ---------------------------------------------------------------------------
# DARBF presets: xi of Table 2; psi as printed in the per-kernel listings
# (the half-cosine uses the listings' 1.36, which the regression also gives;
# the inverse multiquadric of Table 1 uses Table 2's 1.61); support = the
# listings' limit on E.
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class KernelSpec:
    kind: int
    xi: float
    psi: float
    e_max: float
    beta: float = 0.0  # roll-off of the modified kinds (GAUSS_BETA .. SINC_BETA)


# Domain limit U of u = d_M^beta / xi for the modified forms (Table 1): one
# half-cosine lobe, n raised-cosine pulses, n sinc pulses; the Gaussian has no
# limit and keeps the 3-sigma box of the fixed kernels (E <= 9).
def modified_e_max(kind: int, xi: float, beta: float, pulses: int = 1) -> float:
    U = {native.HALF_COS_BETA: 0.5 * math.pi, native.RAISED_COS_BETA: pulses * math.pi,
         native.SINC_BETA: 0.5 * (pulses + 1) * math.pi}.get(kind)
    if U is None:
        return 9.0
    return (xi * U) ** (2.0 / beta)


def modified_kernel(kind: int, xi: float, beta: float, psi: float, pulses: int = 1) -> KernelSpec:
    """A modified DARBF of Table 1 with roll-off ``beta`` and its support of
    ``pulses`` lobes (raised cosine, sinc)."""
    return KernelSpec(kind, xi, psi, modified_e_max(kind, xi, beta, pulses), beta)


KERNELS = {
    "gauss": KernelSpec(native.GAUSS, 2.0, 1.0, 9.0),
    "half_cos": KernelSpec(native.HALF_COS, 18.0 / math.pi, 1.36, 9.0),
    "raised_cos": KernelSpec(native.RAISED_COS, 2.5 / math.pi, 0.655, 6.25),
    "sinc": KernelSpec(native.SINC, 3.0 / math.pi, 1.18, 9.0),
    "imq": KernelSpec(native.IMQ, 1.0, 1.38, 9.0),
    "imq_sqrt": KernelSpec(native.IMQ_SQRT, 1.0, 1.61, 9.0),
    "parabola": KernelSpec(native.PARABOLA, 9.0, 1.3, 9.0),
}
# Modified forms of Table 1 (generic roll-off, several pulses).  psi is the
# marginal-covariance ratio of each form as the correction-factor experiment
# on the GPU (calibrate.calibrate_psi, 1000 covariances, 97^3 grid) measures it.
KERNELS.update({
    # exp(-d_M^4 / 2), the 3-sigma box of the Gaussian
    "gauss_b4": modified_kernel(native.GAUSS_BETA, 2.0, 4.0, 0.349),
    # cos(d_M / xi) on its main lobe, xi = 6/pi: the lobe ends at d_M = 3 like the half-cosine's
    "half_cos_b1": modified_kernel(native.HALF_COS_BETA, 6.0 / math.pi, 1.0, 1.247),
    # the raised cosine of the listings (beta = 1, xi = 2.5/pi) with two pulses: d_M <= 5
    "raised_cos_n2": modified_kernel(native.RAISED_COS_BETA, 2.5 / math.pi, 1.0, 6.205, pulses=2),
    # the modular sinc of the listings (beta = 1, xi = 3/pi) with three pulses: d_M <= 6
    "sinc_n3": modified_kernel(native.SINC_BETA, 3.0 / math.pi, 1.0, 5.676, pulses=3),
})

DEFAULT_OPTS = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, bg=(0.0, 0.0, 0.0))


def n_tiles(width: int, height: int) -> int:
    return ((width + 15) // 16) * ((height + 15) // 16)


def splats_to_device(sp: dict, device="cuda") -> dict:
    out = {k: torch.as_tensor(v).to(device).contiguous() for k, v in sp.items() if k != "sh_degree"}
    out["sh_degree"] = int(sp["sh_degree"])
    return out


def alloc_projected(n: int, device="cuda", dcolor: bool = True) -> dict:
    """Projected records; ``dcolor`` keeps the colour checkpoint the preprocess
    backward reads instead of the SH coefficients (forward-only users skip it)."""
    f = dict(dtype=torch.float32, device=device)
    return dict(xy=torch.empty((n, 2), **f), depth=torch.empty(n, **f),
                radius=torch.empty(n, dtype=torch.int32, device=device),
                extent=torch.empty((n, 2), dtype=torch.int32, device=device), conic_o=torch.empty((n, 4), **f),
                rgb=torch.empty((n, 3), **f), clamped=torch.empty(n, dtype=torch.uint8, device=device),
                dcolor=torch.empty((9, n), **f) if dcolor else None)


@dataclass
class Frame:
    """Buffers of one view: projection, binning and the forward checkpoint."""
    n: int
    width: int
    height: int
    proj: dict
    ws: torch.Tensor
    vals: torch.Tensor
    ranges: torch.Tensor
    k_dev: torch.Tensor
    overflow: torch.Tensor
    image: torch.Tensor
    final_T: torch.Tensor
    last: torch.Tensor
    n_contrib: torch.Tensor | None = None
    keys: torch.Tensor | None = None
    K: int | None = None
    extras: dict = field(default_factory=dict)

    @property
    def capacity(self) -> int:
        return int(self.vals.numel())


def alloc_frame(n: int, width: int, height: int, k_capacity: int, device="cuda", keys: bool = False,
                n_contrib: bool = False, proj: dict | None = None, dcolor: bool = True,
                ws: torch.Tensor | None = None) -> Frame:
    """Buffers of one render.  ``ws``: a bin/sort workspace to use instead of a
    new one (at least the size this frame needs); frames whose bin/sorts run one
    after another on one stream can share it."""
    cap = max(int(k_capacity), 1)
    ws_bytes = native.darb_bin_sort_workspace(n, width, height, cap)
    if ws_bytes == 0:
        raise native.DarbError(native.DARB_ERR_UNSUPPORTED, f"unsupported size n={n} {width}x{height} cap={cap}")
    if ws is not None and ws.numel() < ws_bytes:
        raise ValueError(f"shared workspace of {ws.numel()} bytes, {ws_bytes} needed")
    T = n_tiles(width, height)
    return Frame(
        n=n, width=width, height=height, proj=proj if proj is not None else alloc_projected(n, device, dcolor),
        ws=ws if ws is not None else torch.empty(ws_bytes, dtype=torch.uint8, device=device),
        vals=torch.empty(cap, dtype=torch.int32, device=device),
        ranges=torch.empty((T, 2), dtype=torch.int32, device=device),
        k_dev=torch.zeros(2, dtype=torch.int64, device=device),
        overflow=torch.zeros(4, dtype=torch.int32, device=device),
        image=torch.empty((3, height, width), dtype=torch.float32, device=device),
        final_T=torch.empty((height, width), dtype=torch.float32, device=device),
        last=torch.empty((height, width), dtype=torch.int32, device=device),
        n_contrib=torch.empty((height, width), dtype=torch.int32, device=device) if n_contrib else None,
        keys=torch.empty(cap, dtype=torch.int64, device=device) if keys else None,
    )


def _grow(frame: Frame, K: int, device):
    cap = int(K * 1.15) + 1024
    frame.ws = None
    frame.ws = torch.empty(native.darb_bin_sort_workspace(frame.n, frame.width, frame.height, cap), dtype=torch.uint8,
                           device=device)
    frame.vals = torch.empty(cap, dtype=torch.int32, device=device)
    if frame.keys is not None:
        frame.keys = torch.empty(cap, dtype=torch.int64, device=device)


def bin_sort(frame: Frame, read_k: bool = True, stream=None):
    """Binning + sort into ``frame``; with ``read_k`` the count is read back and
    the capacity grown (and the call repeated) when it was too small."""
    dev = frame.vals.device
    K = native.darb_bin_sort(frame.proj, frame.n, frame.width, frame.height, frame.capacity, frame.ws, frame.keys,
                             frame.vals, frame.ranges, frame.k_dev, frame.overflow, read_k=read_k, stream=stream)
    if read_k and K > frame.capacity:
        _grow(frame, K, dev)
        K = native.darb_bin_sort(frame.proj, frame.n, frame.width, frame.height, frame.capacity, frame.ws,
                                 frame.keys, frame.vals, frame.ranges, frame.k_dev, frame.overflow, read_k=True,
                                 stream=stream)
    frame.K = K
    return K


def render(splats: dict, cam: dict, kernel: KernelSpec, opts: dict | None = None, frame: Frame | None = None,
           k_capacity: int | None = None, read_k: bool = True, keys: bool = False, n_contrib: bool = False,
           zero_g2d: dict | None = None, stream=None) -> Frame:
    """preprocess -> bin/sort -> raster forward.  Returns the frame with the
    image and the checkpoint (final T, last position).  ``zero_g2d``: 2D-gradient
    buffers the raster forward also clears (see render_backward's g2d_zeroed)."""
    opts = opts or DEFAULT_OPTS
    n = int(splats["means"].shape[1])
    W, H = int(cam["width"]), int(cam["height"])
    dev = splats["means"].device
    if frame is None:
        cap = k_capacity if k_capacity is not None else max(4 * n, 1 << 16)
        frame = alloc_frame(n, W, H, cap, dev, keys=keys, n_contrib=n_contrib)
    native.darb_preprocess(cam, kernel, n, splats, frame.proj, stream=stream)
    bin_sort(frame, read_k=read_k, stream=stream)
    native.darb_raster_fwd(frame.proj, n, frame.vals, frame.ranges, frame.overflow, W, H, kernel, opts, frame.image,
                           frame.final_T, frame.last, frame.n_contrib, zero_g2d=zero_g2d, stream=stream)
    return frame


def forward_overlapped(splats: dict, cam: dict, kernel: KernelSpec, frame: Frame, side, opts: dict | None = None,
                       zero_g2d: dict | None = None, main=None):
    """The forward of a training step into a sized ``frame`` with no host sync:
    the preprocess geometry on ``main`` (default: the current stream), then its
    colour part on the ``side`` stream while ``main`` bins and sorts, joined
    before the raster forward.  The results are the bits of ``render``."""
    opts = opts or DEFAULT_OPTS
    main = main if main is not None else torch.cuda.current_stream()
    n = frame.n
    native.darb_preprocess(cam, kernel, n, splats, frame.proj, parts=native.PRE_GEOMETRY, stream=main)
    side.wait_stream(main)
    native.darb_preprocess(cam, kernel, n, splats, frame.proj, parts=native.PRE_COLOUR, stream=side)
    native.darb_bin_sort(frame.proj, n, frame.width, frame.height, frame.capacity, frame.ws, frame.keys, frame.vals,
                         frame.ranges, frame.k_dev, frame.overflow, stream=main)
    main.wait_stream(side)
    native.darb_raster_fwd(frame.proj, n, frame.vals, frame.ranges, frame.overflow, frame.width, frame.height, kernel,
                           opts, frame.image, frame.final_T, frame.last, frame.n_contrib, zero_g2d=zero_g2d,
                           stream=main)
    return frame


def alloc_grads(n: int, sh_degree: int, device="cuda"):
    f = dict(dtype=torch.float32, device=device)
    g2d = dict(xy=torch.empty((n, 2), **f), conic=torch.empty((n, 3), **f), opacity=torch.empty(n, **f),
               rgb=torch.empty((n, 3), **f))
    nb = (sh_degree + 1) ** 2
    g3d = dict(means=torch.empty((3, n), **f), scales=torch.empty((3, n), **f), quats=torch.empty((4, n), **f),
               opacity=torch.empty(n, **f), sh=torch.empty((nb, 3, n), **f))
    return g2d, g3d


def det_workspace(frame: Frame) -> torch.Tensor:
    """Workspace of the deterministic raster backward of ``frame``."""
    nb = native.darb_raster_bwd_workspace(frame.n, frame.width, frame.height, frame.capacity)
    if nb == 0:
        raise native.DarbError(native.DARB_ERR_UNSUPPORTED, "no deterministic workspace for this size")
    return torch.empty(nb, dtype=torch.uint8, device=frame.vals.device)


def render_backward(frame: Frame, dL_dimage: torch.Tensor, splats: dict, cam: dict, kernel: KernelSpec,
                    opts: dict | None = None, grads=None, chain: bool = True, stream=None, deterministic: bool = False,
                    det_ws: torch.Tensor | None = None, g2d_zeroed: bool = False):
    """raster backward (+ the preprocess chain when ``chain``) from the checkpoint.
    ``g2d_zeroed``: grads[0] was cleared by the forward (render's zero_g2d)."""
    opts = opts or DEFAULT_OPTS
    n = frame.n
    if grads is None:
        grads = alloc_grads(n, int(splats["sh_degree"]), frame.image.device)
    g2d, g3d = grads
    if deterministic and det_ws is None:
        det_ws = det_workspace(frame)
    native.darb_raster_bwd(frame.proj, n, frame.vals, frame.ranges, frame.overflow, frame.width, frame.height, kernel,
                           opts, dL_dimage.contiguous(), frame.final_T, frame.last, g2d,
                           cam if chain else None, splats if chain else None, g3d if chain else None,
                           deterministic=deterministic, k_capacity=frame.capacity,
                           ws=det_ws if deterministic else None, g2d_zeroed=g2d_zeroed, stream=stream)
    return g2d, g3d


# ---------------------------------------------------------------------------
# Several views of one scene per step (batched training).
# ---------------------------------------------------------------------------

@dataclass
class MultiFrame:
    """Per-view buffers of a multi-view step (one Frame, 2D-gradient set and
    upstream-gradient image per view)."""
    cams: list
    frames: list
    g2d: list
    dL: list
    det_ws: torch.Tensor | None = None
    side: list | None = None  # side streams of the concurrent per-view bin/sorts

    @property
    def n(self) -> int:
        return self.frames[0].n


def alloc_multiview(n: int, cams: list, capacities: list, device="cuda") -> MultiFrame:
    frames = [alloc_frame(n, int(c["width"]), int(c["height"]), cap, device) for c, cap in zip(cams, capacities)]
    g2d = [alloc_grads(n, 0, device)[0] for _ in cams]
    dL = [torch.empty((3, int(c["height"]), int(c["width"])), dtype=torch.float32, device=device) for c in cams]
    return MultiFrame(cams=list(cams), frames=frames, g2d=g2d, dL=dL)


def multiview_views(mf: MultiFrame, targets: list | None = None, with_dL: bool = False) -> list:
    out = []
    for v, (cam, fr) in enumerate(zip(mf.cams, mf.frames)):
        out.append(dict(cam=cam, proj=fr.proj, k_capacity=fr.capacity, vals=fr.vals, ranges=fr.ranges,
                        overflow_dev=fr.overflow, image=fr.image, final_T=fr.final_T, last=fr.last,
                        n_contrib=fr.n_contrib, dL_dimage=mf.dL[v] if with_dL else None,
                        target=targets[v] if targets is not None else None, grads2d=mf.g2d[v]))
    return out


def multiview_det_workspace(mf: MultiFrame) -> torch.Tensor:
    nb = native.darb_raster_bwd_multi_workspace(multiview_views(mf), mf.n)
    if nb == 0:
        raise native.DarbError(native.DARB_ERR_UNSUPPORTED, "no deterministic workspace for these views")
    return torch.empty(nb, dtype=torch.uint8, device=mf.frames[0].vals.device)


def multiview_overflowed(mf: MultiFrame) -> bool:
    """Reads every view's instance count back (blocking); grows the lists of the
    views that overflowed and returns True when the step must be repeated."""
    again = False
    for fr in mf.frames:
        K = int(fr.k_dev[0].item())
        fr.K = K
        if K > fr.capacity:
            _grow(fr, K, fr.vals.device)
            again = True
    if again:
        mf.det_ws = None
    return again


def multiview_bin_sort(mf: MultiFrame, bin_streams: int = 4, stream=None):
    """Bin/sort of every view.  The views' bin/sorts are independent (each frame
    has its own workspace, lists and counters) and each is a chain of ~20 small,
    latency-bound launches, so with ``bin_streams`` > 1 they run on that many
    side streams (default priority), forked from and joined to ``stream``
    (default: the current stream); the lists are the same either way."""
    n = mf.n
    main = stream if stream is not None else torch.cuda.current_stream()
    k = min(int(bin_streams), len(mf.frames))
    if k <= 1:
        for fr in mf.frames:
            native.darb_bin_sort(fr.proj, n, fr.width, fr.height, fr.capacity, fr.ws, None, fr.vals, fr.ranges,
                                 fr.k_dev, fr.overflow, stream=main)
        return
    if mf.side is None or len(mf.side) < k:
        mf.side = [torch.cuda.Stream(device=mf.frames[0].vals.device) for _ in range(k)]
    side = mf.side[:k]
    for s in side:
        s.wait_stream(main)
    for v, fr in enumerate(mf.frames):
        native.darb_bin_sort(fr.proj, n, fr.width, fr.height, fr.capacity, fr.ws, None, fr.vals, fr.ranges, fr.k_dev,
                             fr.overflow, stream=side[v % k])
    for s in side:
        main.wait_stream(s)


def multiview_step(splats: dict, mf: MultiFrame, targets: list, kernel: KernelSpec, g3d: dict,
                   opts: dict | None = None, loss_kind: int = native.LOSS_L1, fused: bool = True,
                   deterministic: bool = False, stream=None, bin_streams: int = 4):
    """One training step over all views: preprocess (one launch) -> bin/sort per
    view (concurrently on ``bin_streams`` side streams, :func:`multiview_bin_sort`)
    -> raster forward + loss + backward (one fused launch, or forward launch,
    per-view loss and backward launch) -> preprocess backward summed over the
    views (one launch) into ``g3d``.  Nothing is read back; a view whose list
    overflowed is skipped (check with :func:`multiview_overflowed`)."""
    opts = opts or DEFAULT_OPTS
    n = mf.n
    views = multiview_views(mf, targets=targets, with_dL=not fused or deterministic)
    native.darb_preprocess_multi(views, kernel, n, splats, stream=stream)
    multiview_bin_sort(mf, bin_streams, stream=stream)
    if fused and not deterministic:
        native.darb_raster_fwdbwd_multi(views, n, kernel, opts, loss_kind, stream=stream)
    else:
        native.darb_raster_fwd_multi(views, n, kernel, opts, stream=stream)
        for v, fr in enumerate(mf.frames):
            native.darb_image_loss(fr.image, targets[v], fr.width, fr.height, loss_kind, dL_dimage=mf.dL[v],
                                   stream=stream)
        if deterministic and mf.det_ws is None:
            mf.det_ws = multiview_det_workspace(mf)
        native.darb_raster_bwd_multi(views, n, kernel, opts, deterministic=deterministic,
                                     ws=mf.det_ws if deterministic else None, stream=stream)
    native.darb_preprocess_bwd_multi(views, kernel, n, splats, g3d, stream=stream)


def sequential_step(splats: dict, mf: MultiFrame, targets: list, kernel: KernelSpec, g3d: dict,
                    opts: dict | None = None, loss_kind: int = native.LOSS_L1, deterministic: bool = False,
                    det_ws: list | None = None, stream=None):
    """The same step as single-view calls, view after view: preprocess ->
    bin/sort -> raster forward -> loss -> raster backward -> preprocess backward
    accumulated into ``g3d``."""
    opts = opts or DEFAULT_OPTS
    n = mf.n
    for v, (cam, fr) in enumerate(zip(mf.cams, mf.frames)):
        native.darb_preprocess(cam, kernel, n, splats, fr.proj, stream=stream)
        native.darb_bin_sort(fr.proj, n, fr.width, fr.height, fr.capacity, fr.ws, None, fr.vals, fr.ranges, fr.k_dev,
                             fr.overflow, stream=stream)
        native.darb_raster_fwd(fr.proj, n, fr.vals, fr.ranges, fr.overflow, fr.width, fr.height, kernel, opts,
                               fr.image, fr.final_T, fr.last, fr.n_contrib, zero_g2d=mf.g2d[v], stream=stream)
        native.darb_image_loss(fr.image, targets[v], fr.width, fr.height, loss_kind, dL_dimage=mf.dL[v], stream=stream)
        ws = None
        if deterministic:
            ws = det_ws[v] if det_ws is not None else det_workspace(fr)
        native.darb_raster_bwd(fr.proj, n, fr.vals, fr.ranges, fr.overflow, fr.width, fr.height, kernel, opts,
                               mf.dL[v], fr.final_T, fr.last, mf.g2d[v], deterministic=deterministic,
                               k_capacity=fr.capacity, ws=ws, g2d_zeroed=True, stream=stream)
        native.darb_preprocess_bwd(cam, kernel, n, splats, mf.g2d[v], g3d, accumulate=v > 0, stream=stream,
                                   proj=fr.proj)
