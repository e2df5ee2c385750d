"""Helpers shared by the GPU parity tests: run the HIP path (through the C ABI)
on seeded numpy inputs and return numpy results, and the comparison rules."""
from __future__ import annotations

import math

import numpy as np
import torch

import oracle
from paper_2501_12369_amd import native, pipeline

PI = math.pi

# Kernel definitions for the oracle, written from the paper (Table 2 xi, the
# listings' psi and support); the HIP side has its own presets.
ORACLE_KERNELS = {
    "gauss": oracle.KernelSpec(oracle.GAUSS, 2.0, 1.0, 9.0),
    "half_cos": oracle.KernelSpec(oracle.HALF_COS, 18.0 / PI, 1.36, 9.0),
    "raised_cos": oracle.KernelSpec(oracle.RAISED_COS, 2.5 / PI, 0.655, 6.25),
    "sinc": oracle.KernelSpec(oracle.SINC, 3.0 / PI, 1.18, 9.0),
    "imq": oracle.KernelSpec(oracle.IMQ, 1.0, 1.38, 9.0),
    "imq_sqrt": oracle.KernelSpec(oracle.IMQ_SQRT, 1.0, 1.61, 9.0),
    "parabola": oracle.KernelSpec(oracle.PARABOLA, 9.0, 1.3, 9.0),
    # Table 1's modified forms: support u = d_M^beta / xi <= U, i.e. E <= (xi U)^(2/beta)
    "gauss_b4": oracle.KernelSpec(oracle.GAUSS_BETA, 2.0, 0.349, 9.0, 4.0),
    "half_cos_b1": oracle.KernelSpec(oracle.HALF_COS_BETA, 6.0 / PI, 1.247, (6.0 / PI * PI / 2) ** 2, 1.0),
    "raised_cos_n2": oracle.KernelSpec(oracle.RAISED_COS_BETA, 2.5 / PI, 6.205, (2.5 / PI * 2 * PI) ** 2, 1.0),
    "sinc_n3": oracle.KernelSpec(oracle.SINC_BETA, 3.0 / PI, 5.676, (3.0 / PI * 2 * PI) ** 2, 1.0),
}


def decision_rings(name: str) -> int:
    """Level sets per footprint where a pixel's decision can flip: the boundaries
    of the ranges of E in (0, e_max] where o F(E) stays below alpha_min at full
    opacity, plus the support edge when F does not vanish there (the Gaussian's
    jump).  One for a single decaying lobe; a kernel with interior zeros (several
    pulses) adds two per zero.  Ambiguous pixels are capped at 0.1% per ring."""
    k = ORACLE_KERNELS[name]
    E = np.linspace(0.0, k.e_max, 200001)
    low = np.abs(oracle.kernel_values(k.kind, k.xi, E, k.beta)) < 1.0 / 255.0
    rings = int(np.count_nonzero(low[1:] != low[:-1]))
    return rings + (0 if low[-1] else 1)


def oracle_kernel_fp32(name: str) -> oracle.KernelSpec:
    """The oracle's kernel with xi/psi/e_max rounded to FP32, as the GPU receives them."""
    k = ORACLE_KERNELS[name]
    f = lambda v: float(np.float32(v))
    return oracle.KernelSpec(k.kind, f(k.xi), f(k.psi), f(k.e_max), f(k.beta))


def oracle_opts_fp32(opts=None):
    o = dict(pipeline.DEFAULT_OPTS)
    o.update(opts or {})
    f = lambda v: float(np.float32(v))
    return oracle.make_opts(f(o["alpha_min"]), f(o["alpha_max"]), f(o["t_min"]), tuple(f(b) for b in o["bg"]))


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def conic_from_factor(l) -> np.ndarray:
    """(a, b, c) of Q = L^T L in FP64 from factors (l00, l01, l11) [n, 3]."""
    l = np.asarray(l, np.float64)
    return np.stack([l[:, 0] ** 2, l[:, 0] * l[:, 1], l[:, 1] ** 2 + l[:, 2] ** 2], 1)


def projected_to_device(ps: dict) -> dict:
    """The device records: the conic as its factor (what the library stores)."""
    n = len(ps["radius"])
    co = np.concatenate([ps["conic_l"], ps["conic_o"][:, 3:4]], 1).astype(np.float32)
    return dict(xy=dev(ps["xy"]), depth=dev(ps["depth"]), radius=dev(ps["radius"]),
                extent=dev(np.asarray(ps["extent"], np.int32).reshape(n, 2)), conic_o=dev(co),
                rgb=dev(ps["rgb"]), clamped=torch.zeros(max(n, 1), dtype=torch.uint8, device="cuda")[:n])


def oracle_projected(ps: dict) -> dict:
    """The oracle's records: the conic of the same factor the GPU receives."""
    return dict(xy=ps["xy"].astype(np.float64), conic=conic_from_factor(ps["conic_l"]),
                rgb=ps["rgb"].astype(np.float64), depth=ps["depth"].astype(np.float64),
                valid=(ps["radius"] > 0).astype(np.int32))


def gpu_bin_raster(ps: dict, kernel_name: str, opts=None, keys=True, cap=None):
    """bin/sort + raster forward of synthetic projected splats on the GPU."""
    n = len(ps["radius"])
    W, H = ps["width"], ps["height"]
    proj = projected_to_device(ps)
    fr = pipeline.alloc_frame(n, W, H, cap if cap is not None else max(1, 64 * n), "cuda", keys=keys,
                              n_contrib=True, proj=proj)
    K = pipeline.bin_sort(fr, read_k=True)
    k = pipeline.KERNELS[kernel_name]
    native.darb_raster_fwd(fr.proj, n, fr.vals, fr.ranges, fr.overflow, W, H, k, opts or pipeline.DEFAULT_OPTS,
                           fr.image, fr.final_T, fr.last, fr.n_contrib)
    torch.cuda.synchronize()
    return fr, K


def to_np(t):
    return t.detach().cpu().numpy()


def image_pixels(img_chw: np.ndarray) -> np.ndarray:
    """[3, H, W] -> [H*W, 3] in the oracle's pixel order (row-major, x fastest)."""
    return img_chw.reshape(3, -1).T


def last_ids(fr) -> np.ndarray:
    """Per-pixel splat id of the last blended instance (-1 if none)."""
    last = to_np(fr.last).reshape(-1).astype(np.int64) & 0xFFFFFFFF
    vals = to_np(fr.vals).astype(np.int64)
    out = np.full(last.shape, -1, np.int64)
    m = last != 0xFFFFFFFF
    out[m] = vals[last[m]]
    return out


def grad_compare(g_gpu: np.ndarray, g_orc: np.ndarray, rel_l2=1e-3, rel_el=1e-3, abs_frac=1e-4, mask=None):
    """Relative L2 error and the elementwise rule |d| <= rel_el |g| + abs_frac max|g|.
    Returns (ok, rel_l2_error, worst_elementwise_ratio)."""
    a = np.asarray(g_gpu, np.float64)
    b = np.asarray(g_orc, np.float64)
    if mask is not None:
        a = a[mask]
        b = b[mask]
    if b.size == 0:
        return True, 0.0, 0.0
    nb = np.linalg.norm(b)
    l2 = np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)
    tol = rel_el * np.abs(b) + abs_frac * np.max(np.abs(b))
    ratio = np.max(np.abs(a - b) / np.maximum(tol, 1e-30))
    return (l2 <= rel_l2) and (ratio <= 1.0), float(l2), float(ratio)


def ambiguous_zeroed(G_hw3: np.ndarray, margin: np.ndarray, ambig: float) -> np.ndarray:
    """The upstream gradient [m, 3] with the rows of decision-ambiguous pixels
    (oracle margin < ``ambig``) set to zero.  A pixel's backward terms are all
    products with its G, so both sides then give exactly zero there and every
    splat's gradient can be compared without exempting any splat."""
    G = np.array(G_hw3, np.float32, copy=True)
    G[margin < ambig] = 0.0
    return G


def assert_grads(g_gpu: dict, g_orc: dict, names, label="", **tol):
    """Every tensor within the gradient rule: relative L2 and elementwise."""
    for name in names:
        ok, l2, ratio = grad_compare(g_gpu[name], g_orc[name], **tol)
        print(f"  {label}{name:8s} relL2={l2:.2e} worst={ratio:.3f}")
        assert ok, (label, name, l2, ratio)


def assert_records_fp32(proj: dict, o: dict, both: np.ndarray, ulps: int = 1, label: str = ""):
    """The records the library stored (mean2D, depth, conic factor) equal the
    oracle's FP64 projection rounded to FP32 (oracle.records_fp32) within
    ``ulps`` units in the last place, on the splats ``both`` sides kept.  The
    library computes the projection in FP64 and rounds once, so a difference
    appears only where the FP64 value lies within FP64 rounding of an FP32
    rounding boundary."""
    r = oracle.records_fp32(o)
    pairs = {"xy": (to_np(proj["xy"])[both], r["xy"][both]),
             "depth": (to_np(proj["depth"])[both], r["depth"][both]),
             "conic_l": (to_np(proj["conic_o"])[both][:, :3], r["conic_l"][both])}
    for name, (g, ref) in pairs.items():
        ref32 = ref.astype(np.float32)
        d = np.abs(np.asarray(g, np.float32).astype(np.float64) - ref32.astype(np.float64))
        sp = np.spacing(np.abs(ref32)).astype(np.float64)
        print(f"  {label}{name}: {int(np.sum(d > 0))} of {d.size} differ from the rounded oracle, "
              f"worst {np.max(d / sp) if d.size else 0:.1f} ulp")
        assert np.all(d <= ulps * sp), name


def visibility_ambiguous(sp: dict, cam: dict, o: dict, idx, rel: float = 1e-5, rf: float = 3.0) -> np.ndarray:
    """For the splats ``idx`` whose culling differs between the two sides: True
    where a culling decision of the oracle lies within ``rel`` (relative) of its
    threshold -- the near plane, the sign of the 2D determinant, a tile-box
    half-extent rf sqrt(Sigma'_xx) or rf sqrt(Sigma'_yy) at an integer, or an
    edge of the tile box on the image's tile border -- so FP32 rounding may
    take it either way."""
    idx = np.atleast_1d(np.asarray(idx, np.int64))
    V = np.asarray(cam["viewmat"], np.float64)
    mu = np.asarray(sp["means"], np.float64)[:, idx]
    t = V[:3, :3] @ mu + V[:3, 3:4]
    near = float(cam["near_z"])
    out = np.abs(t[2] - near) <= rel * near
    cov = o["cov2d"][idx]
    det = cov[:, 0] * cov[:, 2] - cov[:, 1] ** 2
    out |= np.abs(det) <= rel * np.abs(cov[:, 0] * cov[:, 2])
    rx3 = rf * np.sqrt(np.maximum(cov[:, 0], 0.0))
    ry3 = rf * np.sqrt(np.maximum(cov[:, 2], 0.0))
    for r3 in (rx3, ry3):
        out |= np.abs(r3 - np.round(r3)) <= rel * np.maximum(r3, 1.0)
    RX, RY = np.ceil(rx3), np.ceil(ry3)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = float(cam["fx"]) * t[0] / t[2] + float(cam["cx"])
        v = float(cam["fy"]) * t[1] / t[2] + float(cam["cy"])
    gx, gy = 16 * ((cam["width"] + 15) // 16), 16 * ((cam["height"] + 15) // 16)
    scale = np.abs(u) + np.abs(v) + RX + RY + 1.0
    for e in (u + RX, u - RX - gx, v + RY, v - RY - gy):
        out |= np.abs(e) <= rel * scale
    return out


def assert_extent(ext_gpu, ext_orc, cov, rf: float = 3.0) -> None:
    """Tile-box half-extents [m, 2] of kept splats: equal to the oracle's unless
    rf sqrt(Sigma'_xx) (or _yy) of the oracle's FP64 covariance ``cov`` [m, 3]
    lies within 1e-4 (relative) of an integer, where the two FP64 chains may
    round it to either side."""
    ext_gpu, ext_orc = np.asarray(ext_gpu), np.asarray(ext_orc)
    for j, c in ((0, 0), (1, 2)):
        r = rf * np.sqrt(cov[:, c])
        near_int = np.abs(r - np.round(r)) < 1e-4 * r
        assert np.array_equal(ext_gpu[~near_int, j], ext_orc[~near_int, j]), j
        assert np.all(np.abs(ext_gpu[near_int, j] - ext_orc[near_int, j]) <= 1), j
