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


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_version_and_status_strings(L):
    from paper_2501_12369_amd import native

    assert native.darb_version() == 1
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
