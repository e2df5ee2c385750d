"""Seeded synthetic inputs for the rasterizer and its oracle.

This module only draws random numbers and builds cameras; it holds none of the
rasterizer's arithmetic, and both the HIP path and the oracle consume what it
returns.  All arrays are FP32 (the precision of the boundary); layouts match
the C-ABI: means/scales [3, n], quats [4, n] (w, x, y, z), opacity [n],
sh [(deg+1)^2, 3, n].

Scene recipes follow the workloads of the paper's evaluation (multi-million
splat scenes, SH degree 3; Experimental setup) without its datasets, which are
not available: everything is drawn from numpy's PCG64 with a fixed seed.
"""
from __future__ import annotations

import math

import numpy as np

# Half-width of the range of a degree-0 SH coefficient whose colour is uniform
# in [0, 1]: colour = Y00 * c + 0.5 with Y00 = 1 / (2 sqrt(pi)), so c in [-sqrt(pi), sqrt(pi)].
_SH0_HALF_RANGE = math.sqrt(math.pi)


def look_at(campos, target, up=(0.0, -1.0, 0.0)) -> np.ndarray:
    """World->camera 4x4 (row-major) for a camera at ``campos`` looking at ``target``.

    Camera frame: x right, y down, z forward (world up = -y by default)."""
    campos = np.asarray(campos, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - campos
    z /= np.linalg.norm(z)
    up = np.asarray(up, dtype=np.float64)
    x = np.cross(up, z)
    if np.linalg.norm(x) < 1e-9:  # looking along the up axis
        x = np.cross(np.array([1.0, 0.0, 0.0]), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z], axis=0)  # rows = camera axes in world coordinates
    M = np.eye(4)
    M[:3, :3] = R
    M[:3, 3] = -R @ campos
    return M


def camera(viewmat, campos, fx, fy, cx, cy, width, height, near_z=0.2, jac_clamp=1.3, dilation=0.3) -> dict:
    return dict(viewmat=np.asarray(viewmat, np.float32).reshape(4, 4), campos=np.asarray(campos, np.float32),
                fx=float(np.float32(fx)), fy=float(np.float32(fy)), cx=float(np.float32(cx)),
                cy=float(np.float32(cy)), width=int(width), height=int(height), near_z=float(np.float32(near_z)),
                jac_clamp=float(np.float32(jac_clamp)), dilation=float(np.float32(dilation)))


def _random_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


def _log_uniform(rng, lo, hi, shape):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=shape)).astype(np.float32)


def _splats(means, scales, quats, opacity, sh, deg):
    return dict(means=np.ascontiguousarray(means, np.float32), scales=np.ascontiguousarray(scales, np.float32),
                quats=np.ascontiguousarray(quats, np.float32), opacity=np.ascontiguousarray(opacity, np.float32),
                sh=np.ascontiguousarray(sh, np.float32), sh_degree=int(deg))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def tiny(seed: int = 1, n: int = 64, width: int = 64, height: int = 64, dilation: float = 0.3) -> dict:
    """64 splats, one 64x64 pinhole view (fx = fy = 64, cx = cy = 32), camera at the
    origin looking +z.  Means uniform in [-1,1]^3 shifted to z in [2,4]; scales
    log-uniform in [0.02, 0.2]; random unit quaternions; opacity U[0.1, 0.9];
    degree-0 colours uniform in [0,1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(-1.0, 1.0, size=(3, n))
    means[2] += 3.0
    scales = _log_uniform(rng, 0.02, 0.2, (3, n))
    quats = _random_quats(rng, n)
    opacity = rng.uniform(0.1, 0.9, size=n)
    sh = rng.uniform(-_SH0_HALF_RANGE, _SH0_HALF_RANGE, size=(1, 3, n))
    cam = camera(np.eye(4), np.zeros(3), 64.0 * width / 64, 64.0 * height / 64, width / 2, height / 2, width,
                 height, dilation=dilation)
    return dict(splats=_splats(means, scales, quats, opacity, sh, 0), camera=cam, seed=seed)


def object_scale(seed: int = 2, n: int = 100_000, width: int = 800, height: int = 800) -> dict:
    """100k splats with means in the unit ball, viewed from radius 4 (fx = fy = 1111);
    scales log-uniform in [0.005, 0.05]; opacity U[0.05, 0.99]; SH degree 3 ~ N(0, 0.3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    means = d * rng.uniform(0.0, 1.0, size=n) ** (1.0 / 3.0)
    scales = _log_uniform(rng, 0.005, 0.05, (3, n))
    quats = _random_quats(rng, n)
    opacity = rng.uniform(0.05, 0.99, size=n)
    sh = rng.normal(0.0, 0.3, size=(16, 3, n))
    campos = np.array([0.0, 0.0, -4.0])
    cam = camera(look_at(campos, np.zeros(3)), campos, 1111.0, 1111.0, width / 2, height / 2, width, height)
    return dict(splats=_splats(means, scales, quats, opacity, sh, 3), camera=cam, seed=seed)


def scene_splats(seed: int, n: int, n_clusters: int = 64, box: float = 10.0) -> dict:
    """Scene-scale splats: means from a seeded mixture of anisotropic Gaussian
    clusters in a [-box, box]^3 box (per-axis std log-uniform in [0.3, 3] m, random
    cluster rotation); scales log-uniform in [0.002, 0.5]; opacity Beta(2, 2);
    SH degree 3 ~ N(0, 0.3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(-box, box, size=(n_clusters, 3))
    stds = np.exp(rng.uniform(math.log(0.3), math.log(3.0), size=(n_clusters, 3)))
    rots = []
    for _ in range(n_clusters):
        a = rng.standard_normal((3, 3))
        qm, r = np.linalg.qr(a)
        qm *= np.sign(np.diag(r))
        rots.append(qm)
    rots = np.stack(rots)
    which = rng.integers(0, n_clusters, size=n)
    z = rng.standard_normal((n, 3, 1), dtype=np.float32) * stds[which][:, :, None].astype(np.float32)
    pts = np.matmul(rots[which].astype(np.float32), z)[:, :, 0] + centres[which].astype(np.float32)
    means = np.clip(pts, -box, box).T
    scales = _log_uniform(rng, 0.002, 0.5, (3, n))
    q = rng.standard_normal((4, n), dtype=np.float32)
    quats = q / np.linalg.norm(q, axis=0, keepdims=True)
    opacity = rng.beta(2.0, 2.0, size=n)
    sh = rng.standard_normal((16, 3, n), dtype=np.float32)
    sh *= np.float32(0.3)
    return _splats(means, scales, quats, opacity, sh, 3)


def orbit_camera(rng, width: int, height: int, radius: float = 15.0, hfov_deg: float = 60.0) -> dict:
    """Camera at distance ``radius`` from the origin in a random direction, looking at
    the origin, focal length for the given horizontal field of view."""
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    campos = d * radius
    f = 0.5 * width / math.tan(math.radians(hfov_deg) / 2.0)
    return camera(look_at(campos, np.zeros(3)), campos, f, f, width / 2, height / 2, width, height)


def scene(seed: int = 3, n: int = 3_000_000, width: int = 1297, height: int = 840) -> dict:
    """Scene-scale workload: 3M clustered splats, one 1297x840 view (60 deg HFOV) from
    15 m in a seeded random direction."""
    splats = scene_splats(seed, n)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    cam = orbit_camera(rng, width, height)
    return dict(splats=splats, camera=cam, seed=seed)


SERVING_RESOLUTIONS = ((640, 360), (1280, 720), (1297, 840), (1920, 1080))
SERVING_SCENE_SIZES = (500_000, 1_000_000, 3_000_000, 6_000_000)


def serving_requests(seed: int, n_requests: int, rate_hz: float = 200.0, n_scenes: int = 4) -> list:
    """Poisson arrivals at ``rate_hz``; each request picks a scene and a resolution
    uniformly and a pose uniformly on the radius-15 sphere around the scene."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))
    out = []
    for i in range(n_requests):
        s = int(rng.integers(0, n_scenes))
        w, h = SERVING_RESOLUTIONS[int(rng.integers(0, len(SERVING_RESOLUTIONS)))]
        out.append(dict(arrival=float(t[i]), scene=s, camera=orbit_camera(rng, w, h)))
    return out


def multiview_cameras(seed: int, n_views: int = 8) -> list:
    """Views at uneven resolutions (W ~ U{640..1920}, H ~ U{480..1080})."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cams = []
    for _ in range(n_views):
        w = int(rng.integers(640, 1921))
        h = int(rng.integers(480, 1081))
        cams.append(orbit_camera(rng, w, h))
    return cams


# --------------------------------------------------------------------------
# synthetic projected splats (inputs of the binning and raster stages)
# --------------------------------------------------------------------------

def projected(seed: int, n: int, width: int, height: int, sigma_range=(0.5, 12.0), opacity_range=(0.05, 0.99),
              margin: float = 20.0, depth_range=(1.0, 20.0), culled_frac: float = 0.1, e_max: float = 9.0) -> dict:
    """Random screen-space splats: centre uniform over the image grown by ``margin``,
    footprint std-devs log-uniform in ``sigma_range`` pixels with a random
    orientation, depth uniform, opacity uniform, colour uniform in [0, 1].

    The conic is the inverse of the drawn covariance R diag(s1^2, s2^2) R^T,
    stored as (a, b, c, opacity); ``conic_l`` holds its upper-triangular
    factor (l00, l01, l11), Q = L^T L.  ``radius`` is ceil(3 * max(s1, s2)) + 1
    pixels, a bound on the support E <= 9 of the one-lobe kernels (with a
    larger support ``e_max``: sqrt(e_max) instead of 3); ``extent`` [n, 2] is
    the tile box's half-width and half-height, ceil(3 sqrt(cov_xx)) + 1 and
    ceil(3 sqrt(cov_yy)) + 1 of the drawn covariance (same factor); a fraction
    ``culled_frac`` of splats get radius and extent 0 (culled)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-margin, width + margin, size=n)
    y = rng.uniform(-margin, height + margin, size=n)
    s1 = np.exp(rng.uniform(math.log(sigma_range[0]), math.log(sigma_range[1]), size=n))
    s2 = np.exp(rng.uniform(math.log(sigma_range[0]), math.log(sigma_range[1]), size=n))
    th = rng.uniform(0.0, math.pi, size=n)
    c, s = np.cos(th), np.sin(th)
    # Q = R diag(1/s1^2, 1/s2^2) R^T with R = [[c, -s], [s, c]]
    i1, i2 = 1.0 / s1 ** 2, 1.0 / s2 ** 2
    qa = c * c * i1 + s * s * i2
    qb = c * s * (i1 - i2)
    qc = s * s * i1 + c * c * i2
    opacity = rng.uniform(opacity_range[0], opacity_range[1], size=n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    depth = rng.uniform(depth_range[0], depth_range[1], size=n)
    rf = math.sqrt(max(9.0, e_max))
    radius = (np.ceil(rf * np.maximum(s1, s2)) + 1).astype(np.int32)
    # covariance R diag(s1^2, s2^2) R^T: diagonal entries
    cxx = c * c * s1 ** 2 + s * s * s2 ** 2
    cyy = s * s * s1 ** 2 + c * c * s2 ** 2
    extent = (np.ceil(rf * np.sqrt(np.stack([cxx, cyy], 1))) + 1).astype(np.int32)
    culled = rng.uniform(size=n) < culled_frac
    radius[culled] = 0
    extent[culled] = 0
    l00 = np.sqrt(qa)
    l01 = qb / l00
    l11 = np.sqrt(i1 * i2 / qa)  # c - b^2/a = det Q / a
    f32 = np.float32
    return dict(xy=np.ascontiguousarray(np.stack([x, y], 1), f32), depth=depth.astype(f32), radius=radius,
                extent=np.ascontiguousarray(extent),
                conic_o=np.ascontiguousarray(np.stack([qa, qb, qc, opacity], 1), f32),
                conic_l=np.ascontiguousarray(np.stack([l00, l01, l11], 1), f32),
                rgb=np.ascontiguousarray(rgb, f32), width=int(width), height=int(height))


def upstream_grad(seed: int, width: int, height: int, kind: str = "normal", sparse_pixels: int | None = None):
    """dL/dimage [3, H, W] FP32.  ``normal``: N(0, 1); ``sign``: +-1 (an L1 gradient
    pattern).  With ``sparse_pixels`` only that many random pixels are nonzero;
    returns (G, pixel list [m, 2] of (x, y)) in that case."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "sign":
        G = np.where(rng.uniform(size=(3, height, width)) < 0.5, -1.0, 1.0)
    else:
        G = rng.standard_normal((3, height, width))
    G = G.astype(np.float32)
    if sparse_pixels is None:
        return G
    idx = rng.choice(width * height, size=sparse_pixels, replace=False)
    mask = np.zeros(width * height, bool)
    mask[idx] = True
    G = G * mask.reshape(1, height, width)
    ys, xs = np.divmod(np.sort(idx), width)
    return G.astype(np.float32), np.stack([xs, ys], 1).astype(np.int32)


def covariances(seed: int, m: int, scale_range=(0.5, 2.0)) -> np.ndarray:
    """m random 3D covariances R diag(s^2) R^T of the scale-and-rotation form
    splats use (random rotation, per-axis scales log-uniform in ``scale_range``),
    as [m, 6] FP64 rows (xx, xy, xz, yy, yz, zz)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((m, 6))
    for i in range(m):
        a = rng.standard_normal((3, 3))
        q, r = np.linalg.qr(a)
        q *= np.sign(np.diag(r))
        s = np.exp(rng.uniform(math.log(scale_range[0]), math.log(scale_range[1]), 3))
        S = (q * s ** 2) @ q.T
        out[i] = [S[0, 0], S[0, 1], S[0, 2], S[1, 1], S[1, 2], S[2, 2]]
    return out


# --------------------------------------------------------------------------
# 1D signal reconstruction (the paper's 1D simulations): target pulses and
# initial mixtures
# --------------------------------------------------------------------------

SIGNALS_1D = ("square", "triangle", "gaussian", "half_sine", "sharp_exponential", "parabola", "trapezoid")


def signals1d(m: int = 1024):
    """x in [-1, 1] (m samples) and the seven target pulses of the paper's 1D
    simulations (square, triangle, Gaussian, half-sinusoid, sharp exponential,
    parabolic, trapezoid), each of height 1 centred at 0; FP32."""
    x = np.linspace(-1.0, 1.0, m)
    ax = np.abs(x)
    sig = dict(
        square=(ax <= 0.4).astype(np.float64),
        triangle=np.clip(1.0 - ax / 0.6, 0.0, None),
        gaussian=np.exp(-0.5 * (x / 0.2) ** 2),
        half_sine=np.where(ax <= 0.5, np.cos(np.pi * x), 0.0),
        sharp_exponential=np.exp(-ax / 0.1),
        parabola=np.clip(1.0 - (x / 0.5) ** 2, 0.0, None),
        trapezoid=np.clip((0.7 - ax) / 0.3, 0.0, 1.0),
    )
    return x.astype(np.float32), {k: v.astype(np.float32) for k, v in sig.items()}


def fit1d_init(seed: int, n: int) -> np.ndarray:
    """Initial mixture [3, n]: means uniform in [-0.8, 0.8], log sigma = log 0.15,
    amplitudes 0.3; FP32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = np.sort(rng.uniform(-0.8, 0.8, n))
    return np.stack([mu, np.full(n, math.log(0.15)), np.full(n, 0.3)]).astype(np.float32)
