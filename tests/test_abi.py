"""Host-side checks of the C ABI library (no GPU): it loads, exports every
symbol that include/darb.h declares, and rejects invalid arguments before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "darb.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"DARB_API\s+[\w\s\*]+?\b(darb_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_2501_12369_amd import native

    return native.lib()


def test_header_declares_the_four_stages():
    names = _declared()
    for n in ("darb_preprocess", "darb_bin_sort", "darb_raster_fwd", "darb_raster_bwd", "darb_preprocess_bwd",
              "darb_bin_sort_workspace", "darb_version", "darb_status_string", "darb_last_error"):
        assert n in names


def test_binding_names_match_the_header():
    from paper_2501_12369_amd import native

    assert sorted(native.EXPORTED) == _declared()


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_version_and_status_strings(L):
    from paper_2501_12369_amd import native

    assert native.darb_version() == 7
    assert L.darb_status_string(0) == b"ok"
    assert L.darb_status_string(2) == b"instance capacity exceeded"


def test_invalid_arguments_rejected_on_host(L):
    from paper_2501_12369_amd import native

    cam = native.darb_camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.near_z = 64, 64, 64.0, 64.0, 0.2
    k = native.darb_kernel(1, 18 / 3.141592653589793, 1.36, 9.0)
    sp = native.darb_splats()
    pr = native.darb_projected()
    # null camera
    st = L.darb_preprocess(None, ctypes.byref(k), 10, ctypes.byref(sp), ctypes.byref(pr), None)
    assert st == native.DARB_ERR_INVALID_ARG
    # null splat pointers with n > 0
    st = L.darb_preprocess(ctypes.byref(cam), ctypes.byref(k), 10, ctypes.byref(sp), ctypes.byref(pr), None)
    assert st == native.DARB_ERR_INVALID_ARG and b"null pointer" in L.darb_last_error()
    # unknown kernel kind / e_max above the binning radius
    for bad in (native.darb_kernel(9, 1.0, 1.0, 9.0), native.darb_kernel(1, 1.0, 1.0, 10.0),
                native.darb_kernel(1, -1.0, 1.0, 9.0)):
        st = L.darb_preprocess(ctypes.byref(cam), ctypes.byref(bad), 0, ctypes.byref(sp), ctypes.byref(pr), None)
        assert st == native.DARB_ERR_INVALID_ARG
    # negative n, oversized image
    st = L.darb_preprocess(ctypes.byref(cam), ctypes.byref(k), -1, ctypes.byref(sp), ctypes.byref(pr), None)
    assert st == native.DARB_ERR_INVALID_ARG
    assert L.darb_bin_sort_workspace(10, 4096, 4096, 100) == 0
    assert L.darb_bin_sort_workspace(10, 16, 16 * 9000, 100) == 0  # too many 8x8-tile groups
    assert L.darb_bin_sort_workspace(-1, 64, 64, 100) == 0
    assert L.darb_bin_sort_workspace(1000, 64, 64, -1) == 0
    assert L.darb_bin_sort_workspace(1000, 64, 64, 100) > 0
    # misaligned pointer
    sp2 = native.darb_splats(16 * 1000 + 4, 16 * 1000, 16 * 1000, 16 * 1000, 16 * 1000, 0)
    st = L.darb_preprocess(ctypes.byref(cam), ctypes.byref(k), 10, ctypes.byref(sp2), ctypes.byref(pr), None)
    assert st == native.DARB_ERR_INVALID_ARG and b"aligned" in L.darb_last_error()


def _view(native, w=64, h=64):
    v = native.darb_view()
    v.cam.width, v.cam.height, v.cam.fx, v.cam.fy, v.cam.near_z = w, h, 64.0, 64.0, 0.2
    return v


def test_multiview_and_loss_arguments_rejected_on_host(L):
    from paper_2501_12369_amd import native

    k = native.darb_kernel(1, 18 / 3.141592653589793, 1.36, 9.0)
    o = native.darb_raster_opts(1 / 255, 0.99, 1e-4)
    sp = native.darb_splats()
    arr = (native.darb_view * 17)()
    for i in range(17):
        arr[i] = _view(native)
    # calibration probes: sizes that are not whole float4 runs, negative counts
    assert L.darb_probe_copy(None, None, 6, None) == native.DARB_ERR_INVALID_ARG
    assert L.darb_probe_fill(None, -4, None) == native.DARB_ERR_INVALID_ARG
    ch = native.c_int32(0)
    assert L.darb_probe_fma(None, 8, -1, 0, ctypes.byref(ch), None) == native.DARB_ERR_INVALID_ARG
    assert L.darb_probe_fma(None, 8, 4, 0, ctypes.byref(ch), None) == native.DARB_ERR_INVALID_ARG  # null out
    # preprocess parts outside {1, 2, 3}
    for parts in (0, 4, -1):
        st = L.darb_preprocess_parts(None, ctypes.byref(k), 0, ctypes.byref(sp), None, parts, None)
        assert st == native.DARB_ERR_INVALID_ARG and b"parts" in L.darb_last_error()
    # view count outside [1, 16]
    for nv in (0, 17):
        st = L.darb_preprocess_multi(arr, nv, ctypes.byref(k), 0, ctypes.byref(sp), None)
        assert st == native.DARB_ERR_INVALID_ARG
    # views without projected buffers / lists / outputs
    st = L.darb_preprocess_multi(arr, 2, ctypes.byref(k), 10, ctypes.byref(sp), None)
    assert st == native.DARB_ERR_INVALID_ARG
    st = L.darb_raster_fwd_multi(arr, 2, 10, ctypes.byref(k), ctypes.byref(o), None)
    assert st == native.DARB_ERR_INVALID_ARG and b"null pointer" in L.darb_last_error()
    st = L.darb_raster_fwdbwd_multi(arr, 2, 10, ctypes.byref(k), ctypes.byref(o), 7, None)
    assert st == native.DARB_ERR_INVALID_ARG and b"loss" in L.darb_last_error()
    # a view with an invalid camera
    bad = (native.darb_view * 1)()
    bad[0] = _view(native, w=0)
    st = L.darb_raster_bwd_multi(bad, 1, 0, ctypes.byref(k), ctypes.byref(o), 0, None, 0, None)
    assert st == native.DARB_ERR_INVALID_ARG
    # image loss: bad kind, null image, loss value without workspace
    st = L.darb_image_loss(None, None, 8, 8, 0, None, None, None, 0, None)
    assert st == native.DARB_ERR_INVALID_ARG
    st = L.darb_image_loss(16, 32, 8, 8, 3, None, None, None, 0, None)
    assert st == native.DARB_ERR_INVALID_ARG
    st = L.darb_image_loss(16, 32, 8, 8, 0, None, 48, None, 0, None)
    assert st == native.DARB_ERR_INVALID_ARG


def test_deterministic_workspace_queries(L):
    from paper_2501_12369_amd import native

    assert L.darb_raster_bwd_workspace(1000, 64, 64, 5000) > L.darb_raster_bwd_workspace(1000, 64, 64, 100) > 0
    assert L.darb_raster_bwd_workspace(1000, 64, 64, -1) == 0
    assert L.darb_raster_bwd_workspace(1000, 4096, 4096, 10) == 0
    arr = (native.darb_view * 3)()
    for i in range(3):
        arr[i] = _view(native)
        arr[i].vals, arr[i].ranges, arr[i].k_capacity = 4096, 8192, 1000
    one = L.darb_raster_bwd_multi_workspace(arr, 1, 100)
    two = L.darb_raster_bwd_multi_workspace(arr, 2, 100)
    assert two > one > 0
    # nv * n beyond 32-bit keys
    assert L.darb_raster_bwd_multi_workspace(arr, 2, 0x7FFFFFFF) > 0
    assert L.darb_raster_bwd_multi_workspace(arr, 3, 0x7FFFFFFF) == 0



def test_noalloc_bin_sort_rejects_on_host(L):
    """darb_bin_sort_noalloc checks its arguments and its scratch limit on the
    host before any HIP call (fake aligned addresses: nothing is launched)."""
    from paper_2501_12369_amd import native

    pr = native.darb_projected()
    # null record pointers with n > 0
    st = L.darb_bin_sort_noalloc(ctypes.byref(pr), 10, 64, 64, 100, None, 4096, 8192, 12288, 16384, None, None)
    assert st == native.DARB_ERR_INVALID_ARG and b"null pointer" in L.darb_last_error()
    pr.xy, pr.depth, pr.radius, pr.extent = 16 * 1000, 16 * 2000, 16 * 3000, 16 * 4000
    # null ranges
    st = L.darb_bin_sort_noalloc(ctypes.byref(pr), 10, 64, 64, 100, None, 4096, None, 12288, 16384, None, None)
    assert st == native.DARB_ERR_INVALID_ARG
    # sizes whose workspace exceeds the scratch: rejected with the sizes in the message
    cap = native.NOALLOC_SCRATCH_BYTES // 4
    assert L.darb_bin_sort_workspace(10, 64, 64, cap) > native.NOALLOC_SCRATCH_BYTES
    st = L.darb_bin_sort_noalloc(ctypes.byref(pr), 10, 64, 64, cap, None, 4096, 8192, 12288, 16384, None, None)
    assert st == native.DARB_ERR_UNSUPPORTED and b"scratch" in L.darb_last_error()
    n = 8_000_000
    assert L.darb_bin_sort_workspace(n, 1297, 840, 1000) > native.NOALLOC_SCRATCH_BYTES
    st = L.darb_bin_sort_noalloc(ctypes.byref(pr), n, 1297, 840, 1000, None, 4096, 8192, 12288, 16384, None, None)
    assert st == native.DARB_ERR_UNSUPPORTED and b"scratch" in L.darb_last_error()
    # the scratch holds the serving scenes' smaller sizes
    assert 0 < L.darb_bin_sort_workspace(1_000_000, 1280, 720, 20_000_000) <= native.NOALLOC_SCRATCH_BYTES
