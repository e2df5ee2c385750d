"""FP64 CPU oracle for the DARB-Splatting rasterizer.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the HIP implementation (see ``oracle.c``); both sides only
consume the same seeded inputs.

Functions here are thin ctypes marshalling around ``liboracle.so`` (plain C,
double precision) plus two pure-Python helpers that the paper fixes:

* :func:`fd_grad` -- central finite differences of a scalar loss computed by
  the oracle's forward (checks the analytic backward against the forward);
* :func:`psi_closed_form` in ``psi.py`` -- the covariance ratio of a 3D radial
  kernel's 2D marginal, which reproduces the paper's correction factors.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

GAUSS, HALF_COS, RAISED_COS, SINC, IMQ, IMQ_SQRT, PARABOLA = range(7)
# Table 1's modified forms with a generic roll-off beta (u = d_M^beta / xi)
GAUSS_BETA, HALF_COS_BETA, RAISED_COS_BETA, SINC_BETA = range(7, 11)
LOSS_L1, LOSS_L2 = 0, 1


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
               "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Camera(ctypes.Structure):
    _fields_ = [("viewmat", ctypes.c_double * 16), ("campos", ctypes.c_double * 3),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("near_z", ctypes.c_double), ("jac_clamp", ctypes.c_double), ("dilation", ctypes.c_double)]


class Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("xi", ctypes.c_double), ("psi", ctypes.c_double),
                ("e_max", ctypes.c_double), ("beta", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double), ("t_min", ctypes.c_double),
                ("bg", ctypes.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        d, i32, i64, vp = ctypes.c_double, ctypes.c_int32, ctypes.c_long, ctypes.c_void_p
        L.orc_kernel_value.restype = d
        L.orc_kernel_value.argtypes = [i32, d, d]
        L.orc_kernel_deriv.restype = d
        L.orc_kernel_deriv.argtypes = [i32, d, d]
        L.orc_kernel_value_beta.restype = d
        L.orc_kernel_value_beta.argtypes = [i32, d, d, d]
        L.orc_kernel_deriv_beta.restype = d
        L.orc_kernel_deriv_beta.argtypes = [i32, d, d, d]
        L.orc_kernel_values.argtypes = [i32, d, d, i64, vp, vp]
        L.orc_kernel_derivs.argtypes = [i32, d, d, i64, vp, vp]
        L.orc_sh_basis.argtypes = [vp, vp, vp]
        L.orc_quat_to_rot.argtypes = [vp, vp]
        L.orc_preprocess.argtypes = [vp, vp, i64, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp,
                                     vp]
        L.orc_composite.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, i64, vp,
                                    ctypes.c_int, vp, vp, vp, vp, vp]
        L.orc_composite_bwd.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, i64, vp,
                                        vp, ctypes.c_int, vp, vp, vp, vp]
        L.orc_preprocess_bwd.argtypes = [vp, vp, i64, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp,
                                         vp, vp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_bin.restype = i64
        L.orc_bin.argtypes = [i64, vp, vp, vp, ctypes.c_int, ctypes.c_int, i64, vp, vp, vp]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    lib().orc_set_num_threads(int(n))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# --------------------------------------------------------------------------
# parameter structs
# --------------------------------------------------------------------------

@dataclass
class KernelSpec:
    kind: int
    xi: float
    psi: float
    e_max: float
    beta: float = 0.0  # roll-off of the modified forms (kinds GAUSS_BETA..SINC_BETA)

    def c(self) -> Kernel:
        return Kernel(self.kind, self.xi, self.psi, self.e_max, self.beta)


def make_camera(viewmat, campos, fx, fy, cx, cy, width, height, near_z=0.2, jac_clamp=1.3, dilation=0.3) -> Camera:
    c = Camera()
    vm = np.asarray(viewmat, dtype=np.float64).reshape(16)
    for k in range(16):
        c.viewmat[k] = float(vm[k])
    for k in range(3):
        c.campos[k] = float(campos[k])
    c.fx, c.fy, c.cx, c.cy = float(fx), float(fy), float(cx), float(cy)
    c.width, c.height = int(width), int(height)
    c.near_z, c.jac_clamp, c.dilation = float(near_z), float(jac_clamp), float(dilation)
    return c


def make_opts(alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, bg=(0.0, 0.0, 0.0)) -> Opts:
    o = Opts()
    o.alpha_min, o.alpha_max, o.t_min = float(alpha_min), float(alpha_max), float(t_min)
    for k in range(3):
        o.bg[k] = float(bg[k])
    return o


def camera_from_scene(cam: dict) -> Camera:
    """Camera struct from a scene-generator camera dict (values as FP32 -> FP64)."""
    return make_camera(np.asarray(cam["viewmat"], np.float32).astype(np.float64),
                       np.asarray(cam["campos"], np.float32).astype(np.float64),
                       np.float32(cam["fx"]), np.float32(cam["fy"]), np.float32(cam["cx"]),
                       np.float32(cam["cy"]), cam["width"], cam["height"], np.float32(cam["near_z"]),
                       np.float32(cam["jac_clamp"]), np.float32(cam["dilation"]))


# --------------------------------------------------------------------------
# wrappers
# --------------------------------------------------------------------------

def kernel_value(kind: int, xi: float, E, beta: float = 0.0) -> np.ndarray:
    L = lib()
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    return np.array([L.orc_kernel_value_beta(kind, xi, beta, float(e)) for e in E])


def kernel_deriv(kind: int, xi: float, E, beta: float = 0.0) -> np.ndarray:
    L = lib()
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    return np.array([L.orc_kernel_deriv_beta(kind, xi, beta, float(e)) for e in E])


def kernel_values(kind: int, xi: float, E, beta: float = 0.0) -> np.ndarray:
    """F at every entry of the array E (same shape)."""
    E = _f64(E)
    out = np.empty_like(E)
    lib().orc_kernel_values(kind, xi, beta, E.size, _p(E), _p(out))
    return out


def kernel_derivs(kind: int, xi: float, E, beta: float = 0.0) -> np.ndarray:
    """dF/dE at every entry of the array E (same shape)."""
    E = _f64(E)
    out = np.empty_like(E)
    lib().orc_kernel_derivs(kind, xi, beta, E.size, _p(E), _p(out))
    return out


def sh_basis(d):
    d = _f64(d)
    Y = np.zeros(16)
    dY = np.zeros((16, 3))
    lib().orc_sh_basis(_p(d), _p(Y), _p(dY))
    return Y, dY


def quat_to_rot(q):
    q = _f64(q)
    R = np.zeros(9)
    lib().orc_quat_to_rot(_p(q), _p(R))
    return R.reshape(3, 3)


def preprocess(cam: Camera, k: KernelSpec, means, scales, quats, sh, deg: int) -> dict:
    """means/scales [3,n], quats [4,n], sh [(deg+1)^2, 3, n]."""
    means, scales, quats, sh = _f64(means), _f64(scales), _f64(quats), _f64(sh)
    n = means.shape[1]
    out = dict(xy=np.zeros((n, 2)), depth=np.zeros(n), radius=np.zeros(n, np.int32),
               extent=np.zeros((n, 2), np.int32), conic=np.zeros((n, 3)),
               rgb=np.zeros((n, 3)), clamped=np.zeros(n, np.uint8), visible=np.zeros(n, np.int32),
               cov2d=np.zeros((n, 3)))
    kc = k.c()
    lib().orc_preprocess(ctypes.byref(cam), ctypes.byref(kc), n, _p(means), _p(scales), _p(quats), _p(sh), deg,
                         _p(out["xy"]), _p(out["depth"]), _p(out["radius"]), _p(out["extent"]), _p(out["conic"]),
                         _p(out["rgb"]),
                         _p(out["clamped"]), _p(out["visible"]), _p(out["cov2d"]))
    return out


def full_pixels(width: int, height: int) -> np.ndarray:
    ys, xs = np.meshgrid(np.arange(height, dtype=np.int32), np.arange(width, dtype=np.int32), indexing="ij")
    return np.ascontiguousarray(np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32))


def composite(proj: dict, opac, k: KernelSpec, opts: Opts, width: int, height: int, pix=None,
              use_grid: bool = True) -> dict:
    """Render the listed pixels ([m,2] int (x, y)); all pixels when pix is None.

    ``proj`` holds xy [n,2], conic [n,3], rgb [n,3], depth [n], and either
    ``visible`` or ``valid`` [n] (nonzero = rendered)."""
    xy, conic, rgb, depth = _f64(proj["xy"]), _f64(proj["conic"]), _f64(proj["rgb"]), _f64(proj["depth"])
    valid = np.ascontiguousarray(np.asarray(proj.get("visible", proj.get("valid")), dtype=np.int32))
    opac = _f64(opac)
    n = xy.shape[0]
    if pix is None:
        pix = full_pixels(width, height)
    pix = np.ascontiguousarray(np.asarray(pix, dtype=np.int32))
    m = pix.shape[0]
    out = dict(rgb=np.zeros((m, 3)), T=np.zeros(m), last=np.zeros(m, np.int64), ncontrib=np.zeros(m, np.int32),
               margin=np.zeros(m))
    kc = k.c()
    lib().orc_composite(n, _p(xy), _p(conic), _p(opac), _p(rgb), _p(depth), _p(valid), ctypes.byref(kc),
                        ctypes.byref(opts), width, height, m, _p(pix), int(use_grid), _p(out["rgb"]), _p(out["T"]),
                        _p(out["last"]), _p(out["ncontrib"]), _p(out["margin"]))
    return out


def composite_bwd(proj: dict, opac, k: KernelSpec, opts: Opts, width: int, height: int, G, pix=None,
                  use_grid: bool = True) -> dict:
    """Gradients of sum_p G_p . I_p w.r.t. xy [n,2], conic [n,3] (a, scalar b, c), opacity [n], rgb [n,3]."""
    xy, conic, rgb, depth = _f64(proj["xy"]), _f64(proj["conic"]), _f64(proj["rgb"]), _f64(proj["depth"])
    valid = np.ascontiguousarray(np.asarray(proj.get("visible", proj.get("valid")), dtype=np.int32))
    opac = _f64(opac)
    n = xy.shape[0]
    if pix is None:
        pix = full_pixels(width, height)
    pix = np.ascontiguousarray(np.asarray(pix, dtype=np.int32))
    G = _f64(G).reshape(pix.shape[0], 3)
    out = dict(xy=np.zeros((n, 2)), conic=np.zeros((n, 3)), opacity=np.zeros(n), rgb=np.zeros((n, 3)))
    kc = k.c()
    lib().orc_composite_bwd(n, _p(xy), _p(conic), _p(opac), _p(rgb), _p(depth), _p(valid), ctypes.byref(kc),
                            ctypes.byref(opts), width, height, pix.shape[0], _p(pix), _p(G), int(use_grid),
                            _p(out["xy"]), _p(out["conic"]), _p(out["opacity"]), _p(out["rgb"]))
    return out


def preprocess_bwd(cam: Camera, k: KernelSpec, means, scales, quats, sh, deg: int, g2d: dict) -> dict:
    means, scales, quats, sh = _f64(means), _f64(scales), _f64(quats), _f64(sh)
    n = means.shape[1]
    gxy, gcon, gop, grgb = _f64(g2d["xy"]), _f64(g2d["conic"]), _f64(g2d["opacity"]), _f64(g2d["rgb"])
    out = dict(means=np.zeros((3, n)), scales=np.zeros((3, n)), quats=np.zeros((4, n)), opacity=np.zeros(n),
               sh=np.zeros(sh.shape))
    kc = k.c()
    lib().orc_preprocess_bwd(ctypes.byref(cam), ctypes.byref(kc), n, _p(means), _p(scales), _p(quats), _p(sh), deg,
                             _p(gxy), _p(gcon), _p(gop), _p(grgb), _p(out["means"]), _p(out["scales"]),
                             _p(out["quats"]), _p(out["opacity"]), _p(out["sh"]))
    return out


def bin_sort(xy, extent, depth, width: int, height: int, cap: int | None = None):
    """Binning reference on FP32 xy [n,2], int32 tile-box half-extents [n,2]
    (rx, ry; 0 = culled), FP32 depth [n].

    Returns (K, keys u64[K], vals u32[K], ranges u32[tiles,2])."""
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float32))
    extent = np.ascontiguousarray(np.asarray(extent, dtype=np.int32).reshape(-1, 2))
    depth = np.ascontiguousarray(np.asarray(depth, dtype=np.float32))
    n = xy.shape[0]
    gx, gy = (width + 15) // 16, (height + 15) // 16
    ranges = np.zeros((gx * gy, 2), np.uint32)
    K = lib().orc_bin(n, _p(xy), _p(extent), _p(depth), width, height, 0, None, None, _p(ranges))
    if cap is None:
        cap = K
    keys = np.zeros(max(K, 1), np.uint64)
    vals = np.zeros(max(K, 1), np.uint32)
    K = lib().orc_bin(n, _p(xy), _p(extent), _p(depth), width, height, cap, _p(keys), _p(vals), _p(ranges))
    return K, keys[:K], vals[:K], ranges


# --------------------------------------------------------------------------
# end-to-end helpers
# --------------------------------------------------------------------------

def conic_factor(cov2d) -> np.ndarray:
    """The triangular factor L = [[l00, l01], [0, l11]] of the conic, Q = L^T L,
    from the 2D covariance (c00, c01, c11) [n, 3]: Q = Sigma'^-1, so
    l11 = 1/sqrt(c11), l00 = sqrt(c11/det), l01 = -c01/sqrt(c11 det),
    det = c00 c11 - c01^2 (the conic's storage form in the projected records)."""
    c = np.asarray(cov2d, np.float64)
    det = c[:, 0] * c[:, 2] - c[:, 1] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.stack([np.sqrt(c[:, 2] / det), -c[:, 1] / np.sqrt(c[:, 2] * det), 1.0 / np.sqrt(c[:, 2])], 1)


def records_fp32(proj: dict) -> dict:
    """The projected records as the C ABI stores them, FP32: mean2D, depth and
    colour rounded to FP32, and the conic stored as its factor L (conic_factor)
    with each entry rounded to FP32.  Returned in FP64 for the composite, the
    conic as L^T L of the rounded factor; culled splats keep zeros."""
    vis = np.asarray(proj["visible"]) != 0
    r32 = lambda a: np.asarray(a, np.float64).astype(np.float32).astype(np.float64)
    L = np.zeros((len(vis), 3))
    L[vis] = r32(conic_factor(proj["cov2d"][vis]))
    conic = np.stack([L[:, 0] ** 2, L[:, 0] * L[:, 1], L[:, 1] ** 2 + L[:, 2] ** 2], 1)
    out = dict(proj)
    out.update(xy=r32(proj["xy"]), depth=r32(proj["depth"]), rgb=r32(proj["rgb"]), conic=conic, conic_l=L)
    return out


def render(cam: Camera, k: KernelSpec, opts: Opts, params: dict, pix=None, use_grid=True, fp32_records=False):
    """preprocess + composite.  params: means, scales, quats, opacity, sh, sh_degree.
    fp32_records: composite the records as the C ABI stores them (records_fp32)
    instead of the FP64 projection."""
    proj = preprocess(cam, k, params["means"], params["scales"], params["quats"], params["sh"],
                      params["sh_degree"])
    src = records_fp32(proj) if fp32_records else proj
    img = composite(src, params["opacity"], k, opts, cam.width, cam.height, pix=pix, use_grid=use_grid)
    return proj, img


def render_bwd(cam: Camera, k: KernelSpec, opts: Opts, params: dict, G, pix=None, use_grid=True):
    proj = preprocess(cam, k, params["means"], params["scales"], params["quats"], params["sh"],
                      params["sh_degree"])
    g2d = composite_bwd(proj, params["opacity"], k, opts, cam.width, cam.height, G, pix=pix, use_grid=use_grid)
    g3d = preprocess_bwd(cam, k, params["means"], params["scales"], params["quats"], params["sh"],
                         params["sh_degree"], g2d)
    return proj, g2d, g3d


def loss_linear(cam: Camera, k: KernelSpec, opts: Opts, params: dict, G, pix=None) -> float:
    """L = sum_p G_p . I_p rendered by the oracle (the scalar the FD driver differentiates)."""
    _, img = render(cam, k, opts, params, pix=pix)
    return float(np.sum(np.asarray(G, dtype=np.float64).reshape(-1, 3) * img["rgb"]))


def fd_grad(fun, x: np.ndarray, index: tuple, rel_h: float = 1e-6) -> float:
    """Central difference of scalar ``fun(x)`` w.r.t. ``x[index]``, h = rel_h * max(1, |x|)."""
    x = np.array(x, dtype=np.float64, copy=True)
    x0 = float(x[index])
    h = rel_h * max(1.0, abs(x0))
    x[index] = x0 + h
    fp = fun(x)
    x[index] = x0 - h
    fm = fun(x)
    return (fp - fm) / (2.0 * h)


def image_loss(image, target, kind: int):
    """Photometric loss of a rendered image, the mean over all its values of
    |I - I_t| (L1, the 3DGS photometric term the paper trains with) or
    (I - I_t)^2 (L2), and its gradient dL/dI (same shape; sign(0) = 0), FP64."""
    d = _f64(image) - _f64(target)
    m = d.size
    if kind == LOSS_L1:
        return float(np.sum(np.abs(d)) / m), np.sign(d) / m
    return float(np.sum(d * d) / m), 2.0 * d / m


def render_bwd_views(cams: list, k: KernelSpec, opts: Opts, params: dict, Gs: list, use_grid=True):
    """Gradients of sum_v sum_p G_v,p . I_v,p: every view's render_bwd, summed
    over the views (the parameters are shared)."""
    total = None
    per_view = []
    for cam, G in zip(cams, Gs):
        _, g2d, g3d = render_bwd(cam, k, opts, params, G, use_grid=use_grid)
        per_view.append(g2d)
        total = {kk: v.copy() for kk, v in g3d.items()} if total is None else {kk: total[kk] + g3d[kk] for kk in total}
    return per_view, total


# ---------------------------------------------------------------------------
# Training-step companions (FP64): the L1 + D-SSIM loss of the Backpropagation
# section, one Adam step, the densification statistics.
# ---------------------------------------------------------------------------

SSIM_RADIUS = 5
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_window() -> np.ndarray:
    """The normalised 11-tap Gaussian (sigma 1.5) of the separable SSIM window."""
    d = np.arange(-SSIM_RADIUS, SSIM_RADIUS + 1, dtype=np.float64)
    g = np.exp(-d * d / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def window_filter(img2d) -> np.ndarray:
    """Window-weighted sums of a 2D array with zero padding outside the image."""
    a = _f64(img2d)
    H, W = a.shape
    g = ssim_window()
    r = SSIM_RADIUS
    pad = np.pad(a, r)
    rows = sum(g[t] * pad[:, t:t + W] for t in range(2 * r + 1))
    return sum(g[t] * rows[t:t + H, :] for t in range(2 * r + 1))


def ssim_map(x2d, y2d):
    """Per-pixel SSIM of one channel, and its partial derivatives with respect to
    the window mean of x, the window variance of x and the window covariance."""
    x, y = _f64(x2d), _f64(y2d)
    mx, my = window_filter(x), window_filter(y)
    vx = window_filter(x * x) - mx * mx
    vy = window_filter(y * y) - my * my
    cxy = window_filter(x * y) - mx * my
    n1, n2 = 2 * mx * my + SSIM_C1, 2 * cxy + SSIM_C2
    d1, d2 = mx * mx + my * my + SSIM_C1, vx + vy + SSIM_C2
    S = n1 * n2 / (d1 * d2)
    dS_dmx = 2 * my * n2 / (d1 * d2) - S * 2 * mx / d1
    dS_dvx = -S / d2
    dS_dcxy = 2 * n1 / (d1 * d2)
    return S, dS_dmx, dS_dvx, dS_dcxy, mx, my


def ssim_loss(image, target, lam: float):
    """(1 - lam) mean|I - I_t| + lam (1 - mean SSIM) over a [3, H, W] image, and its
    gradient dL/dI.  The gradient of sum_p SSIM_p with respect to x_q collects,
    through every window containing q, the chain through the window mean, the
    variance E[x^2] - mean^2 and the covariance E[x y] - mean_x mean_y."""
    I, T = _f64(image), _f64(target)
    m = I.size
    ssum = 0.0
    grad = np.zeros_like(I)
    for c in range(I.shape[0]):
        S, A, B, C, mx, my = ssim_map(I[c], T[c])
        ssum += S.sum()
        dsum = window_filter(A - 2 * B * mx - C * my) + 2 * I[c] * window_filter(B) + T[c] * window_filter(C)
        grad[c] = ((1 - lam) * np.sign(I[c] - T[c]) - lam * dsum) / m
    loss = (1 - lam) * np.abs(I - T).sum() / m + lam * (1 - ssum / m)
    return float(loss), grad


def adam_step(param, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (returns new param, m, v), FP64."""
    p, g, m, v = _f64(param), _f64(grad), _f64(m), _f64(v)
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    denom = np.sqrt(v) / np.sqrt(1 - beta2 ** step) + eps
    return p - lr / (1 - beta1 ** step) * m / denom, m, v


def densify_stats(g_xy, radius, grad_accum, count, max_radius):
    """Per splat with radius > 0: accumulate the 2D mean-gradient norm and the
    view count, and keep the largest radius."""
    g = _f64(g_xy).reshape(-1, 2)
    r = np.asarray(radius)
    vis = r > 0
    acc = _f64(grad_accum).copy()
    cnt = np.array(count, dtype=np.int64, copy=True)
    mr = np.array(max_radius, dtype=np.int64, copy=True)
    acc[vis] += np.sqrt((g[vis] ** 2).sum(1))
    cnt[vis] += 1
    mr[vis] = np.maximum(mr[vis], r[vis])
    return acc, cnt, mr
