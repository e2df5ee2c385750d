"""darb_bin_sort_noalloc (the library's own scratch, no workspace argument)
against darb_bin_sort (caller workspace) through the C ABI: keys, values,
ranges, K and N_v bit for bit on two calls in a row, the second smaller than
the first (the scratch keeps the first call's contents), in both store paths
(keys requested, values only), and the oracle's binning on the same inputs."""
import numpy as np
import pytest
import torch

import oracle
from paper_2501_12369_amd import native, pipeline, scenes

from gpu_util import projected_to_device

pytestmark = pytest.mark.gpu


def to_np(t):
    return t.cpu().numpy()


def run_both(ps, keys: bool):
    n = len(ps["radius"])
    W, H = ps["width"], ps["height"]
    K_o, keys_o, vals_o, ranges_o = oracle.bin_sort(ps["xy"], ps["extent"], ps["depth"], W, H)
    cap = max(K_o, 1)
    proj = projected_to_device(ps)
    ref = pipeline.alloc_frame(n, W, H, cap, "cuda", keys=keys, proj=proj)
    out = pipeline.alloc_frame(n, W, H, cap, "cuda", keys=keys, proj=proj)
    # stale values in every output, so a missing store shows
    for fr in (ref, out):
        fr.vals.fill_(-3)
        fr.ranges.fill_(-5)
        fr.k_dev.fill_(-7)
        fr.overflow.fill_(9)
        if fr.keys is not None:
            fr.keys.fill_(-11)
    K_ref = native.darb_bin_sort(ref.proj, n, W, H, cap, ref.ws, ref.keys, ref.vals, ref.ranges, ref.k_dev,
                                 ref.overflow, read_k=True)
    K_na = native.darb_bin_sort_noalloc(out.proj, n, W, H, cap, out.keys, out.vals, out.ranges, out.k_dev,
                                        out.overflow, read_k=True)
    torch.cuda.synchronize()
    assert K_ref == K_o and K_na == K_o
    assert np.array_equal(to_np(out.k_dev), to_np(ref.k_dev))
    assert int(to_np(out.overflow)[0]) == 0
    assert np.array_equal(to_np(out.ranges), to_np(ref.ranges))
    assert np.array_equal(to_np(out.vals)[:K_o], to_np(ref.vals)[:K_o])
    assert np.array_equal(to_np(out.vals)[:K_o].view(np.uint32), vals_o)
    assert np.array_equal(to_np(out.ranges).view(np.uint32), ranges_o)
    if keys:
        assert np.array_equal(to_np(out.keys)[:K_o], to_np(ref.keys)[:K_o])
        assert np.array_equal(to_np(out.keys)[:K_o].view(np.uint64), keys_o)
    return K_o


@pytest.mark.parametrize("keys", [False, True])
def test_noalloc_matches_workspace_call_twice(keys):
    big = scenes.projected(21, 60000, 1920, 1080, sigma_range=(0.3, 40.0))
    big["depth"][::7] = big["depth"][3]  # equal depths keep index order
    small = scenes.projected(22, 777, 333, 211, sigma_range=(0.5, 20.0))
    print(f"noalloc keys={keys}: 60000 splats 1920x1080, then 777 splats 333x211", flush=True)
    K1 = run_both(big, keys)
    K2 = run_both(small, keys)
    assert K1 > 16 * K2 > 0


def test_noalloc_rejects_beyond_scratch_and_reports_overflow():
    # beyond the scratch: a host-side error before any launch
    ps = scenes.projected(23, 64, 64, 64)
    K_o, _, _, _ = oracle.bin_sort(ps["xy"], ps["extent"], ps["depth"], 64, 64)
    assert K_o > 1
    proj = projected_to_device(ps)
    fr = pipeline.alloc_frame(64, 64, 64, K_o, "cuda", proj=proj)
    big_cap = native.NOALLOC_SCRATCH_BYTES  # >= 8 bytes of list per instance: far beyond the scratch
    assert native.darb_bin_sort_workspace(64, 64, 64, big_cap) > native.NOALLOC_SCRATCH_BYTES
    with pytest.raises(native.DarbError) as e:
        native.darb_bin_sort_noalloc(fr.proj, 64, 64, 64, big_cap, None, fr.vals, fr.ranges, fr.k_dev, fr.overflow)
    assert e.value.status == native.DARB_ERR_UNSUPPORTED and "scratch" in str(e.value)
    # capacity overflow on the device, as the workspace call reports it
    assert native.darb_bin_sort_noalloc(fr.proj, 64, 64, 64, K_o - 1, None, fr.vals, fr.ranges, fr.k_dev,
                                        fr.overflow) is None
    torch.cuda.synchronize()
    assert int(to_np(fr.overflow)[0]) == 1 and int(to_np(fr.k_dev)[0]) == K_o
