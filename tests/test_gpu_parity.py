"""Parity of the HIP path (called through the C ABI) with the FP64 oracle.

Stage tests feed both sides the same seeded inputs:
  * bin/sort: synthetic projected splats -> keys, values, ranges, K bit-exact;
  * raster forward: synthetic projected splats -> image within 1e-5 relative
    (+1e-6 absolute), final T within 1e-5, last contributor and count exact,
    on every pixel whose decisions are not within 1e-4 of a threshold;
  * raster backward: the same plus an upstream gradient -> 2D gradients within
    1e-3 (relative L2, and elementwise 1e-3 |g| + 1e-4 max|g|);
  * preprocess / preprocess backward: splat parameters -> projected records /
    3D gradients at the tolerances derived in the design notes.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2501_12369_amd import native, pipeline, scenes

from gpu_util import (assert_extent, ORACLE_KERNELS, ambiguous_zeroed, assert_grads, assert_records_fp32, conic_from_factor,
                      decision_rings, dev,
                      gpu_bin_raster, grad_compare, image_pixels, last_ids, oracle_kernel_fp32, oracle_opts_fp32,
                      oracle_projected, projected_to_device, to_np, visibility_ambiguous)

pytestmark = pytest.mark.gpu

ALL_KERNELS = list(ORACLE_KERNELS)
AMBIG = 2e-5


# ---------------------------------------------------------------- bin / sort

def _values_only_matches(ps, K_o, vals_o, ranges_o):
    # without the optional keys the last level writes the list with its own store path
    fr, K = gpu_bin_raster(ps, "half_cos", keys=False, cap=max(K_o, 1))
    assert K == K_o
    assert np.array_equal(to_np(fr.ranges).view(np.uint32), ranges_o)
    assert np.array_equal(to_np(fr.vals)[:K].view(np.uint32), vals_o)


# (tile grids up to 255 x 255 carry the tile box through the depth sort in 8-bit
# coordinates; 4080 px is the largest such width, 4100 and 4200 px take the
# record gather instead)
@pytest.mark.parametrize("n,W,H,seed", [(0, 64, 48, 1), (1, 16, 16, 2), (500, 200, 150, 3), (3000, 37, 21, 4),
                                        (20000, 640, 360, 5), (5000, 1297, 840, 6), (20000, 4080, 300, 7),
                                        (20000, 4100, 300, 8), (8000, 200, 4200, 9)])
def test_bin_sort_bit_exact(n, W, H, seed):
    print(f"bin_sort n={n} {W}x{H} seed={seed}", flush=True)
    ps = scenes.projected(seed, n, W, H, sigma_range=(0.3, 25.0))
    if n > 10:
        ps["depth"][::5] = ps["depth"][1]  # ties: equal depth keys must keep index order
    K_o, keys_o, vals_o, ranges_o = oracle.bin_sort(ps["xy"], ps["extent"], ps["depth"], W, H)
    fr, K = gpu_bin_raster(ps, "half_cos", keys=True, cap=max(K_o, 1))
    assert K == K_o
    assert int(to_np(fr.k_dev)[0]) == K_o
    assert int(to_np(fr.overflow)[0]) == 0
    assert np.array_equal(to_np(fr.ranges).view(np.uint32), ranges_o)
    assert np.array_equal(to_np(fr.vals)[:K].view(np.uint32), vals_o)
    assert np.array_equal(to_np(fr.keys)[:K].view(np.uint64), keys_o)
    _values_only_matches(ps, K_o, vals_o, ranges_o)


@pytest.mark.parametrize("n,W,H,seed,sigma", [(300, 200, 150, 9, (50.0, 400.0)), (60000, 1920, 1080, 10, (0.3, 60.0))])
def test_bin_sort_bit_exact_large_boxes(n, W, H, seed, sigma):
    # boxes spanning many 8x8-tile groups, and group lists longer than one chunk
    print(f"bin_sort large boxes n={n} {W}x{H} sigma={sigma}", flush=True)
    ps = scenes.projected(seed, n, W, H, sigma_range=sigma)
    K_o, keys_o, vals_o, ranges_o = oracle.bin_sort(ps["xy"], ps["extent"], ps["depth"], W, H)
    fr, K = gpu_bin_raster(ps, "half_cos", keys=True, cap=K_o)
    assert K == K_o
    assert np.array_equal(to_np(fr.ranges).view(np.uint32), ranges_o)
    assert np.array_equal(to_np(fr.vals)[:K].view(np.uint32), vals_o)
    assert np.array_equal(to_np(fr.keys)[:K].view(np.uint64), keys_o)
    _values_only_matches(ps, K_o, vals_o, ranges_o)


def test_bin_sort_all_culled_and_overflow():
    ps = scenes.projected(7, 300, 96, 64)
    ps["radius"][:] = 0
    ps["extent"][:] = 0
    fr, K = gpu_bin_raster(ps, "gauss", cap=16)
    assert K == 0 and np.all(to_np(fr.ranges) == 0)
    assert np.all(to_np(fr.final_T) == 1.0) and np.all(to_np(fr.image) == 0.0)
    # capacity overflow: flag set, K reported, raster writes nothing
    ps = scenes.projected(8, 300, 96, 64)
    K_o, _, _, _ = oracle.bin_sort(ps["xy"], ps["extent"], ps["depth"], 96, 64)
    proj = projected_to_device(ps)
    fr = pipeline.alloc_frame(300, 96, 64, K_o - 1, "cuda", proj=proj)
    # without the readback the call does not block and reports the overflow on the device
    assert native.darb_bin_sort(fr.proj, 300, 96, 64, K_o - 1, fr.ws, None, fr.vals, fr.ranges, fr.k_dev,
                                fr.overflow, read_k=False) is None
    torch.cuda.synchronize()
    assert int(to_np(fr.overflow)[0]) == 1 and int(to_np(fr.k_dev)[0]) == K_o
    fr.image.fill_(-7.0)
    native.darb_raster_fwd(fr.proj, 300, fr.vals, fr.ranges, fr.overflow, 96, 64, pipeline.KERNELS["gauss"],
                           pipeline.DEFAULT_OPTS, fr.image, fr.final_T, fr.last, None)
    torch.cuda.synchronize()
    assert np.all(to_np(fr.image) == -7.0)
    Kr = native.darb_bin_sort(fr.proj, 300, 96, 64, K_o - 1, fr.ws, None, fr.vals, fr.ranges, fr.k_dev, fr.overflow,
                              read_k=True)
    assert Kr == K_o


# ---------------------------------------------------------------- raster forward

def _forward_case(kname, n, W, H, seed, opts=None, sigma=(0.5, 12.0)):
    ps = scenes.projected(seed, n, W, H, sigma_range=sigma, e_max=ORACLE_KERNELS[kname].e_max)
    fr, K = gpu_bin_raster(ps, kname, opts=opts)
    ko = oracle_kernel_fp32(kname)
    oo = oracle_opts_fp32(opts)
    orc = oracle.composite(oracle_projected(ps), ps["conic_o"][:, 3].astype(np.float64), ko, oo, W, H)
    return ps, fr, orc


@pytest.mark.parametrize("kname", ALL_KERNELS)
@pytest.mark.parametrize("n,W,H,seed", [(1500, 200, 150, 11), (400, 37, 45, 12)])
def test_raster_fwd_parity(kname, n, W, H, seed):
    print(f"raster_fwd {kname} n={n} {W}x{H} seed={seed}", flush=True)
    opts = dict(pipeline.DEFAULT_OPTS, bg=(0.1, 0.2, 0.3))
    ps, fr, orc = _forward_case(kname, n, W, H, seed, opts=opts)
    img = image_pixels(to_np(fr.image))
    Tg = to_np(fr.final_T).reshape(-1)
    amb = orc["margin"] < AMBIG
    ok = ~amb
    assert amb.mean() <= 1e-3 * decision_rings(kname), f"ambiguous fraction {amb.mean()}"
    err = np.abs(img - orc["rgb"])
    tol = 1e-5 * np.abs(orc["rgb"]) + 1e-6
    print(f"  max|dI|={err[ok].max():.3e}  worst ratio={np.max(err[ok] / tol[ok]):.3f}  ambiguous={amb.sum()}")
    assert np.all(err[ok] <= tol[ok])
    assert np.all(np.abs(Tg - orc["T"])[ok] <= 1e-5 * np.abs(orc["T"][ok]) + 1e-7)
    assert np.array_equal(last_ids(fr)[ok], orc["last"][ok])
    assert np.array_equal(to_np(fr.n_contrib).reshape(-1)[ok], orc["ncontrib"][ok])
    assert orc["ncontrib"].max() >= 5


def test_raster_fwd_saturating_and_deterministic():
    # many large opaque splats: the transmittance cut and early tile exit matter
    ps = scenes.projected(13, 4000, 160, 96, sigma_range=(2.0, 30.0), opacity_range=(0.5, 0.99))
    fr, _ = gpu_bin_raster(ps, "half_cos")
    img1 = to_np(fr.image).copy()
    fr2, _ = gpu_bin_raster(ps, "half_cos")
    assert np.array_equal(img1, to_np(fr2.image))  # atomic-free forward: bit-identical across runs
    orc = oracle.composite(oracle_projected(ps), ps["conic_o"][:, 3].astype(np.float64),
                           oracle_kernel_fp32("half_cos"), oracle_opts_fp32(), 160, 96)
    ok = orc["margin"] >= AMBIG
    err = np.abs(image_pixels(img1) - orc["rgb"])
    assert np.all(err[ok] <= 1e-5 * np.abs(orc["rgb"][ok]) + 1e-6)
    assert np.mean(orc["T"] < 2e-3) > 0.3  # most pixels saturate


# ---------------------------------------------------------------- raster backward

@pytest.mark.parametrize("kname", ALL_KERNELS)
def test_raster_bwd_parity(kname):
    n, W, H, seed = 1200, 120, 90, 21
    print(f"raster_bwd {kname} n={n} {W}x{H}", flush=True)
    opts = dict(pipeline.DEFAULT_OPTS, bg=(0.3, 0.1, 0.2))
    ps, fr, orc = _forward_case(kname, n, W, H, seed, opts=opts)
    # the upstream gradient is zeroed on decision-ambiguous pixels (both sides), so
    # every splat is compared
    amb = orc["margin"] < AMBIG
    assert amb.mean() <= 1e-3 * decision_rings(kname), f"ambiguous fraction {amb.mean()}"
    Go = ambiguous_zeroed(scenes.upstream_grad(seed + 1, W, H).reshape(3, -1).T, orc["margin"], AMBIG)
    G = np.ascontiguousarray(Go.T.reshape(3, H, W))
    runs = {}
    for det in (False, True, True):
        g2d, _ = pipeline.alloc_grads(n, 0)
        ws = pipeline.det_workspace(fr) if det else None
        native.darb_raster_bwd(fr.proj, n, fr.vals, fr.ranges, fr.overflow, W, H, pipeline.KERNELS[kname], opts,
                               dev(G), fr.final_T, fr.last, g2d, deterministic=det, k_capacity=fr.capacity, ws=ws)
        torch.cuda.synchronize()
        runs.setdefault(det, []).append({k: to_np(v) for k, v in g2d.items()})
    # the deterministic reduction gives the same bits every run
    for k in runs[True][0]:
        assert np.array_equal(runs[True][0][k], runs[True][1][k]), k
    go = oracle.composite_bwd(oracle_projected(ps), ps["conic_o"][:, 3].astype(np.float64),
                              oracle_kernel_fp32(kname), oracle_opts_fp32(opts), W, H, Go.astype(np.float64))
    for det in (False, True):
        assert_grads(runs[det][0], go, ("xy", "conic", "opacity", "rgb"), label=f"det={int(det)} ")


@pytest.mark.parametrize("n,lo,hi", [(700, 512, 1024), (2600, 1024, 1 << 30)])
def test_raster_bwd_long_walks(n, lo, hi):
    """Dense tiles of faint, wide splats: walks of several hundred to a few
    thousand instances, so that the atomic backward shares a tile's walk among
    two (walk > 512) or four (walk > 1024) wavefronts.  The gradients equal
    the oracle's and the deterministic path's within the gradient rule."""
    kname, W, H, seed = "half_cos", 56, 40, 29
    print(f"raster_bwd long walks n={n} {W}x{H}", flush=True)
    opts = dict(pipeline.DEFAULT_OPTS, bg=(0.2, 0.3, 0.1))
    # faint opacities, so that thousands of splats blend before a pixel saturates
    ps = scenes.projected(seed, n, W, H, sigma_range=(6.0, 25.0), opacity_range=(0.005, 0.03))
    fr, _ = gpu_bin_raster(ps, kname, opts=opts)
    orc = oracle.composite(oracle_projected(ps), ps["conic_o"][:, 3].astype(np.float64), oracle_kernel_fp32(kname),
                           oracle_opts_fp32(opts), W, H)
    # the walks (largest checkpointed position + 1 past the tile's start) span the range
    gx, gy = (W + 15) // 16, (H + 15) // 16
    last = to_np(fr.last).reshape(H, W).astype(np.int64) & 0xFFFFFFFF
    lp = np.where(last == 0xFFFFFFFF, 0, last + 1)
    rng_t = to_np(fr.ranges).astype(np.int64).reshape(-1, 2)
    walks = []
    for ty in range(gy):
        for tx in range(gx):
            st, en = rng_t[ty * gx + tx]
            m = min(int(lp[16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16].max()), int(en))
            walks.append(max(m - int(st), 0))
    print(f"  walks {sorted(walks)}")
    assert any(lo < w <= hi for w in walks), walks
    amb = orc["margin"] < AMBIG
    Go = ambiguous_zeroed(scenes.upstream_grad(seed + 1, W, H).reshape(3, -1).T, orc["margin"], AMBIG)
    G = np.ascontiguousarray(Go.T.reshape(3, H, W))
    print(f"  ambiguous pixels {int(amb.sum())} of {amb.size}")
    assert amb.mean() < 0.25
    runs = {}
    for det in (False, True):
        g2d, _ = pipeline.alloc_grads(n, 0)
        ws = pipeline.det_workspace(fr) if det else None
        native.darb_raster_bwd(fr.proj, n, fr.vals, fr.ranges, fr.overflow, W, H, pipeline.KERNELS[kname], opts,
                               dev(G), fr.final_T, fr.last, g2d, deterministic=det, k_capacity=fr.capacity, ws=ws)
        torch.cuda.synchronize()
        runs[det] = {k: to_np(v) for k, v in g2d.items()}
    go = oracle.composite_bwd(oracle_projected(ps), ps["conic_o"][:, 3].astype(np.float64),
                              oracle_kernel_fp32(kname), oracle_opts_fp32(opts), W, H, Go.astype(np.float64))
    for det in (False, True):
        assert_grads(runs[det], go, ("xy", "conic", "opacity", "rgb"), label=f"det={int(det)} ")


@pytest.mark.parametrize("n", [1200, 7])
def test_raster_fwd_clears_g2d(n):
    """zero_g2d: the forward clears the 2D-gradient buffers (also when the
    overflow flag is set) and its own outputs keep their bits; the backward
    told that they are zero (g2d_zeroed) gives the bits of the default call
    (deterministic mode, so that the comparison is exact)."""
    kname, W, H, seed = "half_cos", 120, 90, 23
    print(f"zero_g2d n={n} {W}x{H}", flush=True)
    ps, fr, _ = _forward_case(kname, n, W, H, seed)
    k, opts = pipeline.KERNELS[kname], pipeline.DEFAULT_OPTS
    ref = {name: to_np(getattr(fr, name)).copy() for name in ("image", "final_T", "last")}
    G = dev(scenes.upstream_grad(seed + 1, W, H))
    ws = pipeline.det_workspace(fr)
    g_ref, _ = pipeline.alloc_grads(n, 0)
    native.darb_raster_bwd(fr.proj, n, fr.vals, fr.ranges, fr.overflow, W, H, k, opts, G, fr.final_T, fr.last, g_ref,
                           deterministic=True, k_capacity=fr.capacity, ws=ws)
    g2, _ = pipeline.alloc_grads(n, 0)
    for t in g2.values():
        t.fill_(float("nan"))
    native.darb_raster_fwd(fr.proj, n, fr.vals, fr.ranges, fr.overflow, W, H, k, opts, fr.image, fr.final_T,
                           fr.last, zero_g2d=g2)
    torch.cuda.synchronize()
    for name, v in ref.items():
        assert np.array_equal(to_np(getattr(fr, name)), v), name
    for name, t in g2.items():
        assert not to_np(t).any(), name
    native.darb_raster_bwd(fr.proj, n, fr.vals, fr.ranges, fr.overflow, W, H, k, opts, G, fr.final_T, fr.last, g2,
                           deterministic=True, k_capacity=fr.capacity, ws=ws, g2d_zeroed=True)
    torch.cuda.synchronize()
    for name in g2:
        assert np.array_equal(to_np(g2[name]), to_np(g_ref[name])), name
    # with the overflow flag set the forward composites nothing but still clears
    for t in g2.values():
        t.fill_(1.0)
    fr.image.fill_(-1.0)
    fr.overflow.fill_(1)
    native.darb_raster_fwd(fr.proj, n, fr.vals, fr.ranges, fr.overflow, W, H, k, opts, fr.image, fr.final_T,
                           fr.last, zero_g2d=g2)
    torch.cuda.synchronize()
    fr.overflow.fill_(0)
    assert np.all(to_np(fr.image) == -1.0)
    for name, t in g2.items():
        assert not to_np(t).any(), name


# ---------------------------------------------------------------- preprocess

def _splats_dev(sp):
    return pipeline.splats_to_device(sp)


@pytest.mark.parametrize("n", [0, 1, 37, 257])
def test_preprocess_parts_small(n):
    """Ragged and empty sizes through the two parts (the colour part loops with
    one workgroup per CU): the one-kernel call's bits, and n = 0 is a no-op."""
    sc = scenes.object_scale(seed=11, n=max(n, 1), width=320, height=240)
    sp, cam = sc["splats"], sc["camera"]
    spd = _splats_dev({k: (v[..., :n] if k != "sh_degree" else v) for k, v in sp.items()})
    print(f"preprocess parts n={n}", flush=True)
    k = pipeline.KERNELS["gauss"]
    one, two = pipeline.alloc_projected(n), pipeline.alloc_projected(n)
    native.darb_preprocess(cam, k, n, spd, one)
    native.darb_preprocess(cam, k, n, spd, two, parts=native.PRE_GEOMETRY)
    native.darb_preprocess(cam, k, n, spd, two, parts=native.PRE_COLOUR)
    torch.cuda.synchronize()
    for name in one:
        assert np.array_equal(to_np(one[name]), to_np(two[name])), name


@pytest.mark.parametrize("deg", [3, 1])
def test_preprocess_parts_bits(deg):
    """The geometry and colour parts (the colour on a second stream after an
    event, as in the overlapped step) write the bits of the one-kernel call,
    for every field, culled splats included."""
    sc = scenes.object_scale(seed=5, n=20000, width=320, height=240)
    sp, cam = dict(sc["splats"]), sc["camera"]
    nb = (deg + 1) ** 2
    sp["sh"], sp["sh_degree"] = np.ascontiguousarray(sp["sh"][:nb]), deg
    n = sp["means"].shape[1]
    print(f"preprocess parts deg={deg} n={n}", flush=True)
    spd = _splats_dev(sp)
    k = pipeline.KERNELS["half_cos"]
    one = pipeline.alloc_projected(n)
    native.darb_preprocess(cam, k, n, spd, one)
    two = pipeline.alloc_projected(n)
    for t in two.values():
        t.fill_(7)  # stale values everywhere: every field must be rewritten
    main, side = torch.cuda.current_stream(), torch.cuda.Stream()
    native.darb_preprocess(cam, k, n, spd, two, parts=native.PRE_GEOMETRY)
    side.wait_stream(main)
    native.darb_preprocess(cam, k, n, spd, two, parts=native.PRE_COLOUR, stream=side)
    main.wait_stream(side)
    torch.cuda.synchronize()
    vis = to_np(one["radius"]) > 0
    assert 0.2 < vis.mean() < 1.0  # both kept and culled splats are covered
    for name in one:
        assert np.array_equal(to_np(one[name]), to_np(two[name])), name


@pytest.mark.parametrize("kname", ["gauss", "half_cos", "raised_cos", "raised_cos_n2"])
@pytest.mark.parametrize("which", ["tiny", "object"])
def test_preprocess_parity(kname, which):
    # raised_cos_n2: two pulses, support E <= 25, so radius and tile box use sqrt(25) = 5 for 3
    sc = scenes.tiny(seed=1) if which == "tiny" else scenes.object_scale(seed=2, n=20000, width=800, height=800)
    sp, cam = sc["splats"], sc["camera"]
    n = sp["means"].shape[1]
    print(f"preprocess {kname} {which} n={n}", flush=True)
    proj = pipeline.alloc_projected(n)
    native.darb_preprocess(cam, pipeline.KERNELS[kname], n, _splats_dev(sp), proj)
    torch.cuda.synchronize()
    o = oracle.preprocess(oracle.camera_from_scene(cam), oracle_kernel_fp32(kname), sp["means"], sp["scales"],
                          sp["quats"], sp["sh"], sp["sh_degree"])
    rad = to_np(proj["radius"])
    vis_g = rad > 0
    vis_o = o["visible"] == 1
    both = vis_g & vis_o
    # visibility may differ only where a culling decision is within rounding of its threshold
    diff = np.flatnonzero(vis_g != vis_o)
    print(f"  visibility differs for {len(diff)} of {n}")
    rf = math.sqrt(max(9.0, oracle_kernel_fp32(kname).e_max))
    assert np.all(visibility_ambiguous(sp, cam, o, diff, rf=rf)), diff
    assert both.sum() > 0.3 * vis_o.sum() and both.sum() > 10
    # mean2D, depth and conic factor: the FP64 projection rounded to FP32, within 1 ulp
    assert_records_fp32(proj, o, both)
    co = to_np(proj["conic_o"])[both]
    rgb = to_np(proj["rgb"])[both]
    # colour (FP32 SH evaluation) relative
    assert np.allclose(rgb, o["rgb"][both], rtol=1e-5, atol=1e-6)
    assert np.array_equal(co[:, 3], sp["opacity"][both])
    # radius: exact unless rf sqrt(lambda_max) lies within 1e-4 of an integer
    cov = o["cov2d"][both]
    mid = 0.5 * (cov[:, 0] + cov[:, 2])
    lam = mid + np.sqrt(np.maximum(mid * mid - (cov[:, 0] * cov[:, 2] - cov[:, 1] ** 2), 0))
    r3 = rf * np.sqrt(lam)
    near_int = np.abs(r3 - np.round(r3)) < 1e-4 * r3
    assert np.array_equal(rad[both][~near_int], o["radius"][both][~near_int])
    # tile box: exact unless rf sqrt(Sigma'_xx) or rf sqrt(Sigma'_yy) lies within 1e-4 of an integer
    assert_extent(to_np(proj["extent"])[both], o["extent"][both], cov, rf=rf)
    ext = to_np(proj["extent"])[both]
    assert np.all(ext <= rad[both][:, None]) and np.all(ext >= 1)


def test_preprocess_huge_footprints():
    """Footprints far larger than the image: radius and tile box capped at
    2^30 px on both sides, the splat kept, its box covering the whole grid (the
    records equal the oracle's; no integer conversion overflows)."""
    n = 6
    means = np.array([[0.0] * n, [0.0] * n, [1.0, 2.0, 5.0, 1.0, 3.0, 2.0]], np.float32)
    scales = np.array([[1e7, 1e9, 1e5, 0.01, 1e12, 3.0]] * 3, np.float32)
    quats = np.tile(np.array([[1.0], [0.2], [0.0], [0.0]], np.float32), (1, n))
    sp = dict(means=means, scales=scales, quats=quats, opacity=np.full(n, 0.5, np.float32),
              sh=np.zeros((1, 3, n), np.float32), sh_degree=0)
    cam = scenes.camera(np.eye(4, dtype=np.float32), np.zeros(3, np.float32), 500.0, 500.0, 320.0, 240.0, 640, 480)
    proj = pipeline.alloc_projected(n)
    native.darb_preprocess(cam, pipeline.KERNELS["half_cos"], n, _splats_dev(sp), proj)
    torch.cuda.synchronize()
    o = oracle.preprocess(oracle.camera_from_scene(cam), oracle_kernel_fp32("half_cos"), means, scales, quats,
                          sp["sh"], 0)
    assert (o["visible"] == 1).all() and (to_np(proj["radius"]) > 0).all()
    cap = 1 << 30
    assert to_np(proj["radius"])[4] == cap and (to_np(proj["extent"])[4] == cap).all()
    assert_extent(to_np(proj["extent"]), o["extent"], o["cov2d"])
    # the capped splat covers every tile of the grid
    fr = pipeline.alloc_frame(n, 640, 480, 1 << 16, "cuda", proj=proj)
    K = pipeline.bin_sort(fr, read_k=True)
    K_o, _, _, _ = oracle.bin_sort(to_np(proj["xy"]), to_np(proj["extent"]), to_np(proj["depth"]), 640, 480)
    assert K == K_o and K >= pipeline.n_tiles(640, 480)


@pytest.mark.parametrize("kname,ckpt", [("gauss", False), ("half_cos", False), ("parabola", False),
                                        ("half_cos", True), ("gauss", True)])
def test_preprocess_bwd_parity(kname, ckpt):
    # ckpt: the colour part from the forward's checkpoint (dcolor, clamped) instead of the SH coefficients
    sc = scenes.object_scale(seed=3, n=5000, width=800, height=800)
    sp, cam = sc["splats"], sc["camera"]
    n = sp["means"].shape[1]
    rng = np.random.default_rng(4)
    g2 = dict(xy=rng.standard_normal((n, 2)).astype(np.float32),
              conic=(rng.standard_normal((n, 3)) * 10).astype(np.float32),
              opacity=rng.standard_normal(n).astype(np.float32),
              rgb=rng.standard_normal((n, 3)).astype(np.float32))
    g2d_dev = {k: dev(v) for k, v in g2.items()}
    _, g3d = pipeline.alloc_grads(n, 3)
    proj = None
    if ckpt:
        proj = pipeline.alloc_projected(n)
        native.darb_preprocess(cam, pipeline.KERNELS[kname], n, _splats_dev(sp), proj)
    native.darb_preprocess_bwd(cam, pipeline.KERNELS[kname], n, _splats_dev(sp), g2d_dev, g3d, proj=proj)
    torch.cuda.synchronize()
    go = oracle.preprocess_bwd(oracle.camera_from_scene(cam), oracle_kernel_fp32(kname), sp["means"], sp["scales"],
                               sp["quats"], sp["sh"], 3, {k: v.astype(np.float64) for k, v in g2.items()})
    o = oracle.preprocess(oracle.camera_from_scene(cam), oracle_kernel_fp32(kname), sp["means"], sp["scales"],
                          sp["quats"], sp["sh"], 3)
    vis = o["visible"] == 1
    for name in ("means", "scales", "quats", "opacity", "sh"):
        a = to_np(g3d[name])
        b = go[name]
        ax = -1
        a_v = np.take(a, np.flatnonzero(vis), axis=ax)
        b_v = np.take(b, np.flatnonzero(vis), axis=ax)
        ok, l2, ratio = grad_compare(a_v, b_v, rel_l2=1e-3, rel_el=1e-3, abs_frac=1e-4)
        print(f"  {name:8s} relL2={l2:.2e} worst={ratio:.3f}")
        assert ok, (name, l2, ratio)
        assert np.all(np.take(a, np.flatnonzero(~vis), axis=ax) == 0.0)


# ---------------------------------------------------------------- end to end (tiny)

@pytest.mark.parametrize("kname,dilation", [(k, e) for k in ("gauss", "half_cos") for e in (0.3, 0.0)] +
                         [(k, 0.3) for k in ("gauss_b4", "half_cos_b1", "raised_cos_n2", "sinc_n3")])
def test_end_to_end_tiny(kname, dilation):
    # the modified forms run the whole path too: their tile boxes take the factor
    # sqrt(e_max) beyond E = 9 (two raised-cosine pulses: 5, three sinc pulses: 6)
    sc = scenes.tiny(seed=1, dilation=dilation)
    sp, cam = sc["splats"], sc["camera"]
    n = sp["means"].shape[1]
    W, H = cam["width"], cam["height"]
    print(f"end-to-end tiny {kname} eps={dilation}", flush=True)
    spd = _splats_dev(sp)
    fr = pipeline.render(spd, cam, pipeline.KERNELS[kname], n_contrib=True)
    ocam = oracle.camera_from_scene(cam)
    ko = oracle_kernel_fp32(kname)
    params = {k: v for k, v in sp.items()}
    _, img_o = oracle.render(ocam, ko, oracle_opts_fp32(), params, fp32_records=True)
    # image: 1e-5 relative + 1e-6 on pixels whose decisions are further than 1e-4
    # (relative) from their thresholds
    ok = img_o["margin"] >= 1e-4
    assert ok.mean() > 0.99
    err = np.abs(image_pixels(to_np(fr.image)) - img_o["rgb"])
    tol = 1e-5 * np.abs(img_o["rgb"]) + 1e-6
    print(f"  image max err {err[ok].max():.2e} worst ratio {np.max(err[ok] / tol[ok]):.3f}, ambiguous {(~ok).sum()}")
    assert np.all(err[ok] <= tol[ok])
    # upstream gradient: the mean-L1 gradient of the oracle's image against a random target,
    # zeroed on the ambiguous pixels on both sides
    target = np.random.default_rng(5).uniform(0, 1, (3, H, W)).astype(np.float32)
    _, Go = oracle.image_loss(img_o["rgb"], image_pixels(target), oracle.LOSS_L1)
    Go = ambiguous_zeroed(Go, img_o["margin"], 1e-4)
    G = np.ascontiguousarray(Go.T.reshape(3, H, W))
    g2d, g3d = pipeline.render_backward(fr, dev(G), spd, cam, pipeline.KERNELS[kname])
    torch.cuda.synchronize()
    _, g2o, g3o = oracle.render_bwd(ocam, ko, oracle_opts_fp32(), params, Go.astype(np.float64))
    assert_grads({k: to_np(v) for k, v in g2d.items()}, g2o, ("xy", "conic", "opacity", "rgb"), label="2D ")
    assert_grads({k: to_np(v) for k, v in g3d.items()}, g3o, ("means", "scales", "quats", "opacity", "sh"),
                 label="3D ")


def test_autograd_matches_plain_path():
    from paper_2501_12369_amd.autograd import rasterize

    sc = scenes.object_scale(seed=9, n=20000, width=320, height=240)
    cam = dict(sc["camera"], fx=450.0, fy=450.0, cx=160.0, cy=120.0)
    spd = _splats_dev(sc["splats"])
    params = [spd[k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]
    img = rasterize(*params, cam, "half_cos", sh_degree=3)
    G = torch.randn_like(img)
    (img * G).sum().backward()
    fr = pipeline.render(spd, cam, pipeline.KERNELS["half_cos"])
    g2d, g3d = pipeline.render_backward(fr, G, spd, cam, pipeline.KERNELS["half_cos"])
    torch.cuda.synchronize()
    assert torch.equal(img.detach(), fr.image)
    for p, name in zip(params, ("means", "scales", "quats", "opacity", "sh")):
        rel = (p.grad - g3d[name]).norm() / g3d[name].norm()
        assert rel < 1e-5, (name, float(rel))  # same kernels; atomics may reorder sums


def test_rasterizer_steps_match_plain_path():
    """The buffer-keeping Rasterizer (overlapped forward, 2D gradients cleared
    by the raster forward) over several steps with moving splats: each step's
    image has the plain path's bits and its gradients match."""
    from paper_2501_12369_amd.autograd import Rasterizer

    sc = scenes.object_scale(seed=10, n=20000, width=320, height=240)
    cam = dict(sc["camera"], fx=450.0, fy=450.0, cx=160.0, cy=120.0)
    spd = _splats_dev(sc["splats"])
    r = Rasterizer("half_cos")
    gen = torch.Generator("cuda").manual_seed(3)
    names = ("means", "scales", "quats", "opacity", "sh")
    for step in range(3):
        print(f"rasterizer step {step}", flush=True)
        spd["means"] = spd["means"] + 0.01 * torch.randn(spd["means"].shape, device="cuda", generator=gen)
        params = [spd[k].clone().requires_grad_(True) for k in names]
        img = r(*params, cam, sh_degree=3)
        G = torch.randn(img.shape, device="cuda", generator=gen)
        (img * G).sum().backward()
        fr = pipeline.render(spd, cam, pipeline.KERNELS["half_cos"])
        _, g3d = pipeline.render_backward(fr, G, spd, cam, pipeline.KERNELS["half_cos"])
        torch.cuda.synchronize()
        assert torch.equal(img.detach(), fr.image)
        for p, name in zip(params, names):
            rel = (p.grad - g3d[name]).norm() / g3d[name].norm()
            assert rel < 1e-5, (step, name, float(rel))


def test_rasterize_gradients_match_oracle():
    """The torch.autograd.Function (checkpointed final T and last position; the
    backward recomputes every pair) against the FP64 oracle: the image within
    1e-5 relative + 1e-6, the 3D gradients of a loss sum(G * image) within the
    gradient rule (G zeroed on decision-ambiguous pixels on both sides)."""
    from paper_2501_12369_amd.autograd import Rasterizer, rasterize

    sc = scenes.object_scale(seed=12, n=3000, width=160, height=120)
    sp = sc["splats"]
    cam = dict(sc["camera"], fx=240.0, fy=240.0, cx=80.0, cy=60.0)
    W, H = cam["width"], cam["height"]
    ocam, ko, oo = oracle.camera_from_scene(cam), oracle_kernel_fp32("half_cos"), oracle_opts_fp32()
    _, img_o = oracle.render(ocam, ko, oo, sp, fp32_records=True)
    ok = img_o["margin"] >= 1e-4
    assert ok.mean() > 0.99
    Go = ambiguous_zeroed(scenes.upstream_grad(13, W, H).reshape(3, -1).T, img_o["margin"], 1e-4)
    _, _, g3o = oracle.render_bwd(ocam, ko, oo, sp, Go.astype(np.float64))
    G = dev(np.ascontiguousarray(Go.T.reshape(3, H, W)))
    spd = _splats_dev(sp)
    names = ("means", "scales", "quats", "opacity", "sh")
    R = Rasterizer("half_cos")
    for label, fn in (("rasterize", lambda *p: rasterize(*p, cam, "half_cos", sh_degree=3)),
                      ("Rasterizer", lambda *p: R(*p, cam, sh_degree=3)),
                      ("Rasterizer again", lambda *p: R(*p, cam, sh_degree=3))):
        print(label, flush=True)
        params = [spd[k].clone().requires_grad_(True) for k in names]
        img = fn(*params)
        (img * G).sum().backward()
        torch.cuda.synchronize()
        err = np.abs(image_pixels(to_np(img)) - img_o["rgb"])
        assert np.all(err[ok] <= 1e-5 * np.abs(img_o["rgb"][ok]) + 1e-6)
        assert_grads({k: to_np(p.grad) for k, p in zip(names, params)}, g3o, names, label=f"{label} ")


def test_rasterizer_two_forwards_one_backward():
    """Two views rendered by one Rasterizer before one backward of the summed
    loss: each forward keeps its own checkpoint, and the gradients equal the
    sum of the plain path's per-view gradients."""
    from paper_2501_12369_amd.autograd import Rasterizer

    sc = scenes.object_scale(seed=14, n=20000, width=320, height=240)
    spd = _splats_dev(sc["splats"])
    cam1 = dict(sc["camera"], fx=450.0, fy=450.0, cx=160.0, cy=120.0)
    campos = np.array([0.6, -0.3, -3.9])
    cam2 = scenes.camera(scenes.look_at(campos, np.zeros(3)), campos, 450.0, 450.0, 160.0, 120.0, 320, 240)
    names = ("means", "scales", "quats", "opacity", "sh")
    gen = torch.Generator("cuda").manual_seed(16)
    G1 = torch.randn((3, 240, 320), device="cuda", generator=gen)
    G2 = torch.randn((3, 240, 320), device="cuda", generator=gen)
    kern = pipeline.KERNELS["half_cos"]
    ref_img, ref_g = [], {k: 0 for k in names}
    for cam, G in ((cam1, G1), (cam2, G2)):
        fr = pipeline.render(spd, cam, kern)
        _, g3d = pipeline.render_backward(fr, G, spd, cam, kern)
        torch.cuda.synchronize()
        ref_img.append(fr.image.clone())
        for k in names:
            ref_g[k] = ref_g[k] + g3d[k]
    R = Rasterizer("half_cos")
    for step in range(3):  # the first step allocates the frames, later ones reuse the pool
        print(f"two forwards, step {step}", flush=True)
        params = [spd[k].clone().requires_grad_(True) for k in names]
        img1 = R(*params, cam1, sh_degree=3)
        img2 = R(*params, cam2, sh_degree=3)
        ((img1 * G1).sum() + (img2 * G2).sum()).backward()
        torch.cuda.synchronize()
        assert torch.equal(img1.detach(), ref_img[0]) and torch.equal(img2.detach(), ref_img[1])
        for p, k in zip(params, names):
            rel = float((p.grad - ref_g[k]).norm() / ref_g[k].norm())
            assert rel < 1e-5, (step, k, rel)
    with torch.no_grad():  # a forward without backward returns its frame to the pool at once
        R(*[spd[k] for k in names], cam1, sh_degree=3)
    assert sum(len(v) for v in R._pool.values()) == 2
