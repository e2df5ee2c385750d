"""ctypes binding of libdarb (``include/darb.h``): argument marshalling only.

Each function has the name of the C entry point it calls and takes torch
tensors (device memory) instead of raw pointers; every step of the rasterizer
runs in the HIP library.  There is no fallback: if ``libdarb.so`` is missing
or fails to load, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdarb.so")

c_float, c_int32, c_int64, c_void_p, c_size_t = (ctypes.c_float, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                                  ctypes.c_size_t)

DARB_OK, DARB_ERR_INVALID_ARG, DARB_ERR_CAPACITY, DARB_ERR_HIP, DARB_ERR_UNSUPPORTED = range(5)
GAUSS, HALF_COS, RAISED_COS, SINC, IMQ, IMQ_SQRT, PARABOLA = range(7)
GAUSS_BETA, HALF_COS_BETA, RAISED_COS_BETA, SINC_BETA = range(7, 11)  # Table 1's modified forms, generic beta
LOSS_L1, LOSS_L2 = 0, 1
MAX_VIEWS = 16
LOSS_WS_BYTES = 4096
NOALLOC_SCRATCH_BYTES = 256 << 20  # DARB_NOALLOC_SCRATCH_BYTES: scratch of darb_bin_sort_noalloc

EXPORTED = ("darb_version", "darb_status_string", "darb_last_error", "darb_preprocess", "darb_preprocess_parts", "darb_preprocess_cam_dev",
            "darb_bin_sort_workspace", "darb_bin_sort", "darb_bin_sort_noalloc", "darb_fit1d", "darb_psi_calibrate_workspace",
            "darb_psi_calibrate", "darb_raster_fwd", "darb_raster_bwd",
            "darb_raster_bwd_workspace", "darb_preprocess_bwd", "darb_image_loss", "darb_preprocess_multi",
            "darb_raster_fwd_multi", "darb_preprocess_multi_cam_dev", "darb_raster_bwd_multi", "darb_raster_bwd_multi_workspace",
            "darb_raster_fwdbwd_multi", "darb_preprocess_bwd_multi", "darb_ssim_loss_workspace", "darb_ssim_loss",
            "darb_adam", "darb_densify_stats", "darb_probe_copy", "darb_probe_fill", "darb_probe_fma")
MAX_ADAM_GROUPS = 8


class DarbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


class darb_camera(ctypes.Structure):
    _fields_ = [("viewmat", c_float * 16), ("campos", c_float * 3), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("width", c_int32), ("height", c_int32), ("near_z", c_float),
                ("jac_clamp", c_float), ("dilation", c_float)]


class darb_kernel(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("xi", c_float), ("psi", c_float), ("e_max", c_float), ("beta", c_float)]


class darb_raster_opts(ctypes.Structure):
    _fields_ = [("alpha_min", c_float), ("alpha_max", c_float), ("t_min", c_float), ("bg", c_float * 3)]


class darb_splats(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("scales", c_void_p), ("quats", c_void_p), ("opacity", c_void_p),
                ("sh", c_void_p), ("sh_degree", c_int32)]


class darb_projected(ctypes.Structure):
    _fields_ = [("xy", c_void_p), ("depth", c_void_p), ("radius", c_void_p), ("extent", c_void_p),
                ("conic_o", c_void_p), ("rgb", c_void_p), ("clamped", c_void_p), ("dcolor", c_void_p)]


class darb_grads2d(ctypes.Structure):
    _fields_ = [("xy", c_void_p), ("conic", c_void_p), ("opacity", c_void_p), ("rgb", c_void_p)]


class darb_grads3d(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("scales", c_void_p), ("quats", c_void_p), ("opacity", c_void_p),
                ("sh", c_void_p)]


class darb_view(ctypes.Structure):
    _fields_ = [("cam", darb_camera), ("proj", darb_projected), ("k_capacity", c_int64), ("vals", c_void_p),
                ("ranges", c_void_p), ("overflow_dev", c_void_p), ("image", c_void_p), ("final_T", c_void_p),
                ("last", c_void_p), ("n_contrib", c_void_p), ("dL_dimage", c_void_p), ("target", c_void_p),
                ("grads2d", darb_grads2d)]


class darb_adam_group(ctypes.Structure):
    _fields_ = [("param", c_void_p), ("grad", c_void_p), ("m", c_void_p), ("v", c_void_p), ("n", c_int64),
                ("lr", c_float)]


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded library; raises if it is not built (there is no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise DarbError(DARB_ERR_UNSUPPORTED,
                            f"{_LIB_PATH} is not built; run `python -m paper_2501_12369_amd.build`")
        L = ctypes.CDLL(_LIB_PATH)
        L.darb_version.restype = c_int32
        L.darb_status_string.restype = ctypes.c_char_p
        L.darb_status_string.argtypes = [c_int32]
        L.darb_last_error.restype = ctypes.c_char_p
        P = ctypes.POINTER
        L.darb_preprocess.restype = c_int32
        L.darb_preprocess.argtypes = [P(darb_camera), P(darb_kernel), c_int64, P(darb_splats), P(darb_projected),
                                      c_void_p]
        L.darb_preprocess_parts.restype = c_int32
        L.darb_preprocess_parts.argtypes = [P(darb_camera), P(darb_kernel), c_int64, P(darb_splats),
                                            P(darb_projected), c_int32, c_void_p]
        L.darb_preprocess_cam_dev.restype = c_int32
        L.darb_preprocess_cam_dev.argtypes = [c_void_p, c_int32, c_int32, P(darb_kernel), c_int64, P(darb_splats),
                                              P(darb_projected), c_void_p]
        L.darb_bin_sort_workspace.restype = c_size_t
        L.darb_bin_sort_workspace.argtypes = [c_int64, c_int32, c_int32, c_int64]
        L.darb_bin_sort.restype = c_int32
        L.darb_bin_sort.argtypes = [P(darb_projected), c_int64, c_int32, c_int32, c_int64, c_void_p, c_size_t,
                                    c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, P(c_int64), c_void_p]
        L.darb_bin_sort_noalloc.restype = c_int32
        L.darb_bin_sort_noalloc.argtypes = [P(darb_projected), c_int64, c_int32, c_int32, c_int64, c_void_p, c_void_p,
                                            c_void_p, c_void_p, c_void_p, P(c_int64), c_void_p]
        L.darb_fit1d.restype = c_int32
        L.darb_fit1d.argtypes = [P(darb_kernel), c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_int32, c_int32, P(c_float), c_float, c_float, c_float, c_void_p, c_void_p]
        L.darb_psi_calibrate_workspace.restype = c_size_t
        L.darb_psi_calibrate_workspace.argtypes = [c_int32, c_int32]
        L.darb_psi_calibrate.restype = c_int32
        L.darb_psi_calibrate.argtypes = [P(darb_kernel), c_int32, c_void_p, c_int32, c_void_p, c_size_t, c_void_p,
                                         c_void_p, c_void_p]
        L.darb_raster_fwd.restype = c_int32
        L.darb_raster_fwd.argtypes = [P(darb_projected), c_int64, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                      P(darb_kernel), P(darb_raster_opts), c_void_p, c_void_p, c_void_p, c_void_p,
                                      P(darb_grads2d), c_void_p]
        L.darb_raster_bwd.restype = c_int32
        L.darb_raster_bwd.argtypes = [P(darb_projected), c_int64, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                      P(darb_kernel), P(darb_raster_opts), c_void_p, c_void_p, c_void_p,
                                      P(darb_grads2d), c_int32, P(darb_camera), P(darb_splats), P(darb_grads3d),
                                      c_int32, c_int64, c_void_p, c_size_t, c_void_p]
        L.darb_raster_bwd_workspace.restype = c_size_t
        L.darb_raster_bwd_workspace.argtypes = [c_int64, c_int32, c_int32, c_int64]
        L.darb_probe_copy.restype = c_int32
        L.darb_probe_copy.argtypes = [c_void_p, c_void_p, c_int64, c_void_p]
        L.darb_probe_fill.restype = c_int32
        L.darb_probe_fill.argtypes = [c_void_p, c_int64, c_void_p]
        L.darb_probe_fma.restype = c_int32
        L.darb_probe_fma.argtypes = [c_void_p, c_int64, c_int32, c_int32, P(c_int32), c_void_p]
        L.darb_preprocess_bwd.restype = c_int32
        L.darb_preprocess_bwd.argtypes = [P(darb_camera), P(darb_kernel), c_int64, P(darb_splats), P(darb_projected),
                                          P(darb_grads2d), P(darb_grads3d), c_int32, c_void_p]
        L.darb_image_loss.restype = c_int32
        L.darb_image_loss.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                      c_size_t, c_void_p]
        L.darb_preprocess_multi.restype = c_int32
        L.darb_preprocess_multi.argtypes = [P(darb_view), c_int32, P(darb_kernel), c_int64, P(darb_splats), c_void_p]
        L.darb_preprocess_multi_cam_dev.restype = c_int32
        L.darb_preprocess_multi_cam_dev.argtypes = [P(darb_view), c_int32, c_void_p, P(darb_kernel), c_int64,
                                                    P(darb_splats), c_void_p]
        L.darb_raster_fwd_multi.restype = c_int32
        L.darb_raster_fwd_multi.argtypes = [P(darb_view), c_int32, c_int64, P(darb_kernel), P(darb_raster_opts),
                                            c_void_p]
        L.darb_raster_bwd_multi.restype = c_int32
        L.darb_raster_bwd_multi.argtypes = [P(darb_view), c_int32, c_int64, P(darb_kernel), P(darb_raster_opts),
                                            c_int32, c_void_p, c_size_t, c_void_p]
        L.darb_raster_bwd_multi_workspace.restype = c_size_t
        L.darb_raster_bwd_multi_workspace.argtypes = [P(darb_view), c_int32, c_int64]
        L.darb_raster_fwdbwd_multi.restype = c_int32
        L.darb_raster_fwdbwd_multi.argtypes = [P(darb_view), c_int32, c_int64, P(darb_kernel), P(darb_raster_opts),
                                               c_int32, c_void_p]
        L.darb_preprocess_bwd_multi.restype = c_int32
        L.darb_preprocess_bwd_multi.argtypes = [P(darb_view), c_int32, P(darb_kernel), c_int64, P(darb_splats),
                                                P(darb_grads3d), c_void_p]
        L.darb_ssim_loss_workspace.restype = c_size_t
        L.darb_ssim_loss_workspace.argtypes = [c_int32, c_int32]
        L.darb_ssim_loss.restype = c_int32
        L.darb_ssim_loss.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_float, c_void_p, c_void_p, c_void_p,
                                     c_size_t, c_void_p]
        L.darb_adam.restype = c_int32
        L.darb_adam.argtypes = [P(darb_adam_group), c_int32, c_int32, c_float, c_float, c_float, c_void_p]
        L.darb_densify_stats.restype = c_int32
        L.darb_densify_stats.argtypes = [P(darb_grads2d), c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != DARB_OK:
        L = lib()
        msg = L.darb_last_error().decode()
        raise DarbError(status, f"{where}: {L.darb_status_string(status).decode()}: {msg}")


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"tensor must live on the GPU, got {t.device}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


# ---------------------------------------------------------------------------
# struct builders
# ---------------------------------------------------------------------------

def camera_struct(cam: dict) -> darb_camera:
    c = darb_camera()
    vm = [float(v) for v in torch.as_tensor(cam["viewmat"], dtype=torch.float64).reshape(16).tolist()]
    for i in range(16):
        c.viewmat[i] = vm[i]
    cp = [float(v) for v in torch.as_tensor(cam["campos"], dtype=torch.float64).reshape(3).tolist()]
    for i in range(3):
        c.campos[i] = cp[i]
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.near_z = float(cam.get("near_z", 0.2))
    c.jac_clamp = float(cam.get("jac_clamp", 1.3))
    c.dilation = float(cam.get("dilation", 0.3))
    return c


def kernel_struct(k) -> darb_kernel:
    return darb_kernel(int(k.kind), float(k.xi), float(k.psi), float(k.e_max), float(getattr(k, "beta", 0.0)))


def opts_struct(o: dict | None = None) -> darb_raster_opts:
    o = o or {}
    s = darb_raster_opts()
    s.alpha_min = float(o.get("alpha_min", 1.0 / 255.0))
    s.alpha_max = float(o.get("alpha_max", 0.99))
    s.t_min = float(o.get("t_min", 1e-4))
    bg = o.get("bg", (0.0, 0.0, 0.0))
    for i in range(3):
        s.bg[i] = float(bg[i])
    return s


def splats_struct(sp: dict) -> darb_splats:
    return darb_splats(_ptr(sp["means"]), _ptr(sp["scales"]), _ptr(sp["quats"]), _ptr(sp["opacity"]),
                       _ptr(sp["sh"]), int(sp["sh_degree"]))


def projected_struct(p: dict) -> darb_projected:
    return darb_projected(_ptr(p["xy"]), _ptr(p["depth"]), _ptr(p["radius"]), _ptr(p["extent"]),
                          _ptr(p.get("conic_o")), _ptr(p.get("rgb")), _ptr(p.get("clamped")), _ptr(p.get("dcolor")))


def grads2d_struct(g: dict) -> darb_grads2d:
    return darb_grads2d(_ptr(g["xy"]), _ptr(g["conic"]), _ptr(g["opacity"]), _ptr(g["rgb"]))


def grads3d_struct(g: dict) -> darb_grads3d:
    return darb_grads3d(_ptr(g["means"]), _ptr(g["scales"]), _ptr(g["quats"]), _ptr(g["opacity"]), _ptr(g["sh"]))


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def darb_version() -> int:
    return int(lib().darb_version())


PRE_GEOMETRY, PRE_COLOUR = 1, 2


def darb_preprocess(cam: dict, kernel, n: int, splats: dict, proj: dict, stream=None, parts: int = 3):
    """parts: PRE_GEOMETRY, PRE_COLOUR or both (3, the single-kernel call)."""
    c, k, s, p = camera_struct(cam), kernel_struct(kernel), splats_struct(splats), projected_struct(proj)
    if parts == 3:
        _check(lib().darb_preprocess(ctypes.byref(c), ctypes.byref(k), n, ctypes.byref(s), ctypes.byref(p),
                                     _stream(stream)), "darb_preprocess")
    else:
        _check(lib().darb_preprocess_parts(ctypes.byref(c), ctypes.byref(k), n, ctypes.byref(s), ctypes.byref(p),
                                           int(parts), _stream(stream)), "darb_preprocess_parts")


def camera_bytes(cam: dict) -> bytes:
    """The darb_camera struct of ``cam`` as raw bytes (for a device camera buffer)."""
    return bytes(camera_struct(cam))


CAMERA_NBYTES = ctypes.sizeof(darb_camera)


def darb_preprocess_cam_dev(cam_dev, width: int, height: int, kernel, n: int, splats: dict, proj: dict,
                            stream=None):
    """``cam_dev``: a device uint8 tensor of CAMERA_NBYTES holding a darb_camera."""
    if cam_dev.numel() * cam_dev.element_size() < CAMERA_NBYTES:
        raise ValueError("camera buffer too small")
    k, s, p = kernel_struct(kernel), splats_struct(splats), projected_struct(proj)
    _check(lib().darb_preprocess_cam_dev(_ptr(cam_dev), width, height, ctypes.byref(k), n, ctypes.byref(s),
                                         ctypes.byref(p), _stream(stream)), "darb_preprocess_cam_dev")


def darb_bin_sort_workspace(n: int, width: int, height: int, k_capacity: int) -> int:
    return int(lib().darb_bin_sort_workspace(n, width, height, k_capacity))


def darb_bin_sort(proj: dict, n: int, width: int, height: int, k_capacity: int, ws, keys, vals, ranges, k_dev,
                  overflow_dev, read_k: bool = False, stream=None):
    """Returns K when ``read_k`` (blocking readback), else None."""
    p = projected_struct(proj)
    kh = c_int64(0)
    st = lib().darb_bin_sort(ctypes.byref(p), n, width, height, k_capacity, _ptr(ws), ws.numel() * ws.element_size(),
                             _ptr(keys), _ptr(vals), _ptr(ranges), _ptr(k_dev), _ptr(overflow_dev),
                             ctypes.byref(kh) if read_k else None, _stream(stream))
    if read_k and st == DARB_ERR_CAPACITY:
        return int(kh.value)
    _check(st, "darb_bin_sort")
    return int(kh.value) if read_k else None


def darb_bin_sort_noalloc(proj: dict, n: int, width: int, height: int, k_capacity: int, keys, vals, ranges, k_dev,
                          overflow_dev, read_k: bool = False, stream=None):
    """darb_bin_sort on the library's own scratch (no workspace argument).
    Returns K when ``read_k`` (blocking readback), else None."""
    p = projected_struct(proj)
    kh = c_int64(0)
    st = lib().darb_bin_sort_noalloc(ctypes.byref(p), n, width, height, k_capacity, _ptr(keys), _ptr(vals),
                                     _ptr(ranges), _ptr(k_dev), _ptr(overflow_dev),
                                     ctypes.byref(kh) if read_k else None, _stream(stream))
    if read_k and st == DARB_ERR_CAPACITY:
        return int(kh.value)
    _check(st, "darb_bin_sort_noalloc")
    return int(kh.value) if read_k else None


def darb_fit1d(kernel, batch: int, n_comp: int, m: int, x, target, params, adam_m, adam_v, steps: int, step0: int,
               lr, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, loss=None, stream=None):
    k = kernel_struct(kernel)
    lr3 = (c_float * 3)(*[float(v) for v in lr])
    _check(lib().darb_fit1d(ctypes.byref(k), batch, n_comp, m, _ptr(x), _ptr(target), _ptr(params), _ptr(adam_m),
                            _ptr(adam_v), steps, step0, lr3, beta1, beta2, eps, _ptr(loss), _stream(stream)),
           "darb_fit1d")


def darb_psi_calibrate_workspace(m: int, grid_n: int) -> int:
    return int(lib().darb_psi_calibrate_workspace(m, grid_n))


def darb_psi_calibrate(kernel, m: int, sigma, grid_n: int, ws, cov2, fit=None, stream=None):
    k = kernel_struct(kernel)
    _check(lib().darb_psi_calibrate(ctypes.byref(k), m, _ptr(sigma), grid_n, _ptr(ws), _nbytes(ws), _ptr(cov2),
                                    _ptr(fit), _stream(stream)), "darb_psi_calibrate")


def darb_raster_fwd(proj: dict, n: int, vals, ranges, overflow_dev, width: int, height: int, kernel, opts: dict,
                    image, final_T, last, n_contrib=None, zero_g2d: dict | None = None, stream=None):
    p, k, o = projected_struct(proj), kernel_struct(kernel), opts_struct(opts)
    z = grads2d_struct(zero_g2d) if zero_g2d is not None else None
    _check(lib().darb_raster_fwd(ctypes.byref(p), n, _ptr(vals), _ptr(ranges), _ptr(overflow_dev), width, height,
                                 ctypes.byref(k), ctypes.byref(o), _ptr(image), _ptr(final_T), _ptr(last),
                                 _ptr(n_contrib), ctypes.byref(z) if z is not None else None, _stream(stream)),
           "darb_raster_fwd")


def _nbytes(t) -> int:
    return 0 if t is None else t.numel() * t.element_size()


def darb_raster_bwd(proj: dict, n: int, vals, ranges, overflow_dev, width: int, height: int, kernel, opts: dict,
                    dL_dimage, final_T, last, g2d: dict, cam: dict | None = None, splats: dict | None = None,
                    g3d: dict | None = None, deterministic: bool = False, k_capacity: int = 0, ws=None,
                    g2d_zeroed: bool = False, stream=None):
    p, k, o = projected_struct(proj), kernel_struct(kernel), opts_struct(opts)
    g2 = grads2d_struct(g2d)
    if g3d is not None:
        c, s, g3 = camera_struct(cam), splats_struct(splats), grads3d_struct(g3d)
        cref, sref, g3ref = ctypes.byref(c), ctypes.byref(s), ctypes.byref(g3)
    else:
        cref = sref = g3ref = None
    _check(lib().darb_raster_bwd(ctypes.byref(p), n, _ptr(vals), _ptr(ranges), _ptr(overflow_dev), width, height,
                                 ctypes.byref(k), ctypes.byref(o), _ptr(dL_dimage), _ptr(final_T), _ptr(last),
                                 ctypes.byref(g2), 1 if g2d_zeroed else 0, cref, sref, g3ref, 1 if deterministic else 0,
                                 int(k_capacity),
                                 _ptr(ws), _nbytes(ws), _stream(stream)), "darb_raster_bwd")


def darb_raster_bwd_workspace(n: int, width: int, height: int, k_capacity: int) -> int:
    return int(lib().darb_raster_bwd_workspace(n, width, height, k_capacity))


def darb_preprocess_bwd(cam: dict, kernel, n: int, splats: dict, g2d: dict, g3d: dict, accumulate: bool = False,
                        stream=None, proj: dict | None = None):
    """``proj``: the records darb_preprocess wrote for this camera; with its
    ``dcolor`` (and ``clamped``) the colour part uses that checkpoint."""
    c, k, s = camera_struct(cam), kernel_struct(kernel), splats_struct(splats)
    g2, g3 = grads2d_struct(g2d), grads3d_struct(g3d)
    p = projected_struct(proj) if proj is not None else None
    _check(lib().darb_preprocess_bwd(ctypes.byref(c), ctypes.byref(k), n, ctypes.byref(s),
                                     ctypes.byref(p) if p is not None else None, ctypes.byref(g2), ctypes.byref(g3),
                                     1 if accumulate else 0, _stream(stream)), "darb_preprocess_bwd")


def darb_image_loss(image, target, width: int, height: int, loss_kind: int, dL_dimage=None, loss_dev=None, ws=None,
                    stream=None):
    _check(lib().darb_image_loss(_ptr(image), _ptr(target), width, height, int(loss_kind), _ptr(dL_dimage),
                                 _ptr(loss_dev), _ptr(ws), _nbytes(ws), _stream(stream)), "darb_image_loss")


def view_struct(v: dict) -> darb_view:
    """``v``: camera dict under "cam" plus any of the darb_view buffers (tensors)."""
    s = darb_view()
    s.cam = camera_struct(v["cam"])
    if v.get("proj") is not None:
        s.proj = projected_struct(v["proj"])
    s.k_capacity = int(v.get("k_capacity", 0))
    for name in ("vals", "ranges", "overflow_dev", "image", "final_T", "last", "n_contrib", "dL_dimage", "target"):
        setattr(s, name, _ptr(v.get(name)))
    if v.get("grads2d") is not None:
        s.grads2d = grads2d_struct(v["grads2d"])
    return s


def views_array(views: list):
    if not 1 <= len(views) <= MAX_VIEWS:
        raise ValueError(f"between 1 and {MAX_VIEWS} views")
    arr = (darb_view * len(views))()
    for i, v in enumerate(views):
        arr[i] = view_struct(v)
    return arr


def darb_preprocess_multi(views: list, kernel, n: int, splats: dict, stream=None):
    a, k, s = views_array(views), kernel_struct(kernel), splats_struct(splats)
    _check(lib().darb_preprocess_multi(a, len(views), ctypes.byref(k), n, ctypes.byref(s), _stream(stream)),
           "darb_preprocess_multi")


def darb_preprocess_multi_cam_dev(views: list, cams_dev, kernel, n: int, splats: dict, stream=None):
    """darb_preprocess_multi with view v's camera read from cams_dev (device bytes
    holding len(views) darb_camera structs)."""
    a, k, s = views_array(views), kernel_struct(kernel), splats_struct(splats)
    _check(lib().darb_preprocess_multi_cam_dev(a, len(views), _ptr(cams_dev), ctypes.byref(k), n, ctypes.byref(s),
                                               _stream(stream)), "darb_preprocess_multi_cam_dev")


def darb_raster_fwd_multi(views: list, n: int, kernel, opts: dict, stream=None):
    a, k, o = views_array(views), kernel_struct(kernel), opts_struct(opts)
    _check(lib().darb_raster_fwd_multi(a, len(views), n, ctypes.byref(k), ctypes.byref(o), _stream(stream)),
           "darb_raster_fwd_multi")


def darb_raster_bwd_multi_workspace(views: list, n: int) -> int:
    return int(lib().darb_raster_bwd_multi_workspace(views_array(views), len(views), n))


def darb_raster_bwd_multi(views: list, n: int, kernel, opts: dict, deterministic: bool = False, ws=None,
                          stream=None):
    a, k, o = views_array(views), kernel_struct(kernel), opts_struct(opts)
    _check(lib().darb_raster_bwd_multi(a, len(views), n, ctypes.byref(k), ctypes.byref(o), 1 if deterministic else 0,
                                       _ptr(ws), _nbytes(ws), _stream(stream)), "darb_raster_bwd_multi")


def darb_raster_fwdbwd_multi(views: list, n: int, kernel, opts: dict, loss_kind: int, stream=None):
    a, k, o = views_array(views), kernel_struct(kernel), opts_struct(opts)
    _check(lib().darb_raster_fwdbwd_multi(a, len(views), n, ctypes.byref(k), ctypes.byref(o), int(loss_kind),
                                          _stream(stream)), "darb_raster_fwdbwd_multi")


def darb_preprocess_bwd_multi(views: list, kernel, n: int, splats: dict, g3d: dict, stream=None):
    a, k, s, g3 = views_array(views), kernel_struct(kernel), splats_struct(splats), grads3d_struct(g3d)
    _check(lib().darb_preprocess_bwd_multi(a, len(views), ctypes.byref(k), n, ctypes.byref(s), ctypes.byref(g3),
                                           _stream(stream)), "darb_preprocess_bwd_multi")


def darb_ssim_loss_workspace(width: int, height: int) -> int:
    return int(lib().darb_ssim_loss_workspace(width, height))


def darb_ssim_loss(image, target, width: int, height: int, lam: float, dL_dimage, loss_dev=None, ws=None,
                   stream=None):
    _check(lib().darb_ssim_loss(_ptr(image), _ptr(target), width, height, float(lam), _ptr(dL_dimage),
                                _ptr(loss_dev), _ptr(ws), _nbytes(ws), _stream(stream)), "darb_ssim_loss")


def darb_adam(groups: list, step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, stream=None):
    """``groups``: dicts with param, grad, m, v (tensors of equal size) and lr."""
    if not 1 <= len(groups) <= MAX_ADAM_GROUPS:
        raise ValueError(f"between 1 and {MAX_ADAM_GROUPS} groups")
    arr = (darb_adam_group * len(groups))()
    for i, g in enumerate(groups):
        n = g["param"].numel()
        for k in ("grad", "m", "v"):
            if g[k].numel() != n:
                raise ValueError(f"group {i}: {k} has {g[k].numel()} values, param has {n}")
        arr[i] = darb_adam_group(_ptr(g["param"]), _ptr(g["grad"]), _ptr(g["m"]), _ptr(g["v"]), n, float(g["lr"]))
    _check(lib().darb_adam(arr, len(groups), int(step), float(beta1), float(beta2), float(eps), _stream(stream)),
           "darb_adam")


def darb_densify_stats(g2d: dict, radius, n: int, grad_accum, count, max_radius=None, stream=None):
    g = grads2d_struct(g2d)
    _check(lib().darb_densify_stats(ctypes.byref(g), _ptr(radius), n, _ptr(grad_accum), _ptr(count),
                                    _ptr(max_radius), _stream(stream)), "darb_densify_stats")


# ---------------------------------------------------------------------------
# Calibration probes (measured ceilings beside the published peaks).
# ---------------------------------------------------------------------------

def darb_probe_copy(src, dst, stream=None):
    _check(lib().darb_probe_copy(_ptr(src), _ptr(dst), src.numel(), _stream(stream)), "darb_probe_copy")


def darb_probe_fill(dst, stream=None):
    _check(lib().darb_probe_fill(_ptr(dst), dst.numel(), _stream(stream)), "darb_probe_fill")


def darb_probe_fma(out, iters: int, stream=None) -> int:
    """FMA chains over out.numel() lanes (FP64 when out is float64); returns the
    number of chains per lane."""
    chains = c_int32(0)
    _check(lib().darb_probe_fma(_ptr(out), out.numel(), int(iters), 1 if out.dtype == torch.float64 else 0,
                                ctypes.byref(chains), _stream(stream)), "darb_probe_fma")
    return int(chains.value)

