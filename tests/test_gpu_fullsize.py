"""Parity at the full workload sizes, in the launch configuration the benchmark
times (the plain render + render_backward path):

  * object scale (100k splats, 800x800, half-cosine): the image on sampled
    pixels against the oracle, and the 3D gradients of 32 random visible splats
    against central finite differences of the oracle's forward (each difference
    renders only the pixels the splat can touch; a difference taken at two step
    sizes that disagree marks a decision flip and the element is skipped);
  * scene scale (3M splats, 1297x840, half-cosine and Gaussian): the image on
    sampled pixels, and -- with an upstream gradient that is nonzero only on a
    set of sampled pixels, so the oracle's per-splat sums are exact -- the 2D
    and 3D gradients of every splat.
Pixels whose oracle decisions sit within 1e-3 (relative) of a threshold are
left out of the samples, so both sides take the same decisions.

The 3D gradients of scale and rotation of a needle-like footprint are small
residuals of the conic gradient along the needle (ill-conditioned: an FP32
chain errs by about eps_32 kappa, kappa = lambda_max / lambda_min of the 2D
covariance); the library runs that chain in FP64.  Every splat is held to
1e-3; the needle-like ones (kappa > 1000: 118 of 1690 half-cosine and 394 of
9057 Gaussian splats that the sampled pixels reach) are also reported apart.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2501_12369_amd import pipeline, scenes

from gpu_util import dev, grad_compare, oracle_kernel_fp32, oracle_opts_fp32, to_np

pytestmark = pytest.mark.gpu

G3 = ("means", "scales", "quats", "opacity", "sh")


def _sample_pixels(rng, W, H, m):
    idx = np.sort(rng.choice(W * H, size=m, replace=False))
    ys, xs = np.divmod(idx, W)
    return np.stack([xs, ys], 1).astype(np.int32)


def _image_at(img_chw, pix):
    return img_chw[:, pix[:, 1], pix[:, 0]].T


def _unambiguous(ocam, ko, oo, params, pix):
    _, img = oracle.render(ocam, ko, oo, params, pix=pix)
    keep = img["margin"] >= 1e-3
    return pix[keep], img["rgb"][keep]


def test_object_scale_image_and_fd_gradients():
    print("full size: object 100k 800x800 half_cos", flush=True)
    sc = scenes.object_scale(seed=2)
    sp, cam = sc["splats"], sc["camera"]
    W, H = cam["width"], cam["height"]
    kern = pipeline.KERNELS["half_cos"]
    spd = pipeline.splats_to_device(sp)
    fr = pipeline.render(spd, cam, kern)
    G = scenes.upstream_grad(21, W, H)
    _, g3d = pipeline.render_backward(fr, dev(G), spd, cam, kern)
    torch.cuda.synchronize()
    img = to_np(fr.image)
    ocam, ko, oo = oracle.camera_from_scene(cam), oracle_kernel_fp32("half_cos"), oracle_opts_fp32()
    params = {k: v for k, v in sp.items()}
    rng = np.random.default_rng(22)
    pix, ref = _unambiguous(ocam, ko, oo, params, _sample_pixels(rng, W, H, 6000))
    err = np.abs(_image_at(img, pix) - ref)
    print(f"  image: {len(pix)} pixels, max err {err.max():.2e}")
    assert np.all(err <= 1e-4 * np.abs(ref) + 1e-5)

    proj = oracle.preprocess(ocam, ko, sp["means"], sp["scales"], sp["quats"], sp["sh"], 3)
    vis = np.flatnonzero(proj["visible"] == 1)
    chosen = rng.choice(vis, size=32, replace=False)
    Gpix = G.transpose(1, 2, 0)  # [H, W, 3]
    checks = [("means", (0,)), ("means", (1,)), ("means", (2,)), ("scales", (0,)), ("scales", (2,)),
              ("quats", (1,)), ("opacity", ()), ("sh", (0, 0)), ("sh", (5, 1))]
    a_all, b_all = [], []
    skipped = 0
    for k in chosen:
        # pixels the splat can touch before and after a small perturbation
        u, v = proj["xy"][k]
        R = int(proj["radius"][k]) + 3
        x0, x1 = max(int(u) - R, 0), min(int(u) + R + 1, W)
        y0, y1 = max(int(v) - R, 0), min(int(v) + R + 1, H)
        if x1 <= x0 or y1 <= y0:
            continue
        ys, xs = np.mgrid[y0:y1, x0:x1]
        pix_k = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)
        Gk = Gpix[pix_k[:, 1], pix_k[:, 0]].astype(np.float64)
        for name, sub in checks:
            idx = sub + (k,)

            def loss(x, name=name):
                p = dict(params)
                p[name] = x
                _, im = oracle.render(ocam, ko, oo, p, pix=pix_k)
                return float(np.sum(Gk * im["rgb"]))

            x = np.asarray(params[name], np.float64)
            f1 = oracle.fd_grad(loss, x, idx, rel_h=1e-6)
            f2 = oracle.fd_grad(loss, x, idx, rel_h=5e-7)
            if abs(f1 - f2) > 1e-4 * max(abs(f1), abs(f2)) + 1e-9:
                skipped += 1  # a decision flipped inside the difference
                continue
            a_all.append(float(to_np(g3d[name])[idx]))
            b_all.append(f1)
    a, b = np.array(a_all), np.array(b_all)
    print(f"  FD: {len(b)} elements checked, {skipped} skipped")
    assert len(b) >= 0.9 * 32 * len(checks)
    ok, l2, ratio = grad_compare(a, b, rel_l2=1e-3, rel_el=1e-3, abs_frac=1e-4)
    print(f"  FD relL2={l2:.2e} worst={ratio:.3f}")
    assert ok, (l2, ratio)


@pytest.mark.parametrize("kname", ["half_cos", "gauss"])
def test_scene_scale_sampled_image_and_sparse_gradients(kname):
    print(f"full size: scene 3M 1297x840 {kname}", flush=True)
    sc = scenes.scene(seed=3)
    sp, cam = sc["splats"], sc["camera"]
    W, H = cam["width"], cam["height"]
    kern = pipeline.KERNELS[kname]
    spd = pipeline.splats_to_device(sp)
    fr = pipeline.render(spd, cam, kern)
    torch.cuda.synchronize()
    img = to_np(fr.image)
    ocam, ko, oo = oracle.camera_from_scene(cam), oracle_kernel_fp32(kname), oracle_opts_fp32()
    params = {k: v for k, v in sp.items()}
    rng = np.random.default_rng(31)
    pix, ref = _unambiguous(ocam, ko, oo, params, _sample_pixels(rng, W, H, 4000))
    err = np.abs(_image_at(img, pix) - ref)
    print(f"  image: {len(pix)} pixels, max err {err.max():.2e}")
    assert np.all(err <= 1e-4 * np.abs(ref) + 1e-5)
    # upstream gradient on the sampled pixels only
    Gs = rng.standard_normal((len(pix), 3)).astype(np.float32)
    G = np.zeros((3, H, W), np.float32)
    G[:, pix[:, 1], pix[:, 0]] = Gs.T
    g2d, g3d = pipeline.render_backward(fr, dev(G), spd, cam, kern)
    torch.cuda.synchronize()
    proj = oracle.preprocess(ocam, ko, sp["means"], sp["scales"], sp["quats"], sp["sh"], 3)
    g2o = oracle.composite_bwd(proj, sp["opacity"], ko, oo, W, H, Gs.astype(np.float64), pix=pix)
    g3o = oracle.preprocess_bwd(ocam, ko, sp["means"], sp["scales"], sp["quats"], sp["sh"], 3, g2o)
    touched = np.flatnonzero(np.abs(g2o["opacity"]) + np.abs(g2o["rgb"]).sum(1) > 0)
    print(f"  splats with gradient: {len(touched)}")
    assert len(touched) > 1000
    for name in ("xy", "conic", "opacity", "rgb"):
        ok, l2, ratio = grad_compare(to_np(g2d[name]), g2o[name], rel_l2=1e-3)
        print(f"  2D {name:8s} relL2={l2:.2e} worst={ratio:.3f}")
        assert l2 <= 1e-3, (name, l2)
    cov = proj["cov2d"]
    mid = 0.5 * (cov[:, 0] + cov[:, 2])
    rad = np.sqrt(np.maximum(mid * mid - (cov[:, 0] * cov[:, 2] - cov[:, 1] ** 2), 0.0))
    kappa = (mid + rad) / np.maximum(mid - rad, 1e-30)
    well = (kappa <= 1000.0) | (proj["visible"] != 1)
    print(f"  needle-like splats among those with gradient: {int((~well[touched]).sum())}")
    for name in G3:
        a, b = to_np(g3d[name]), g3o[name]
        l2w = np.linalg.norm((a - b)[..., well]) / np.linalg.norm(b[..., well])
        l2n = np.linalg.norm((a - b)[..., ~well]) / max(np.linalg.norm(b[..., ~well]), 1e-30)
        print(f"  3D {name:8s} relL2 kappa<=1000 {l2w:.2e}, beyond {l2n:.2e}")
        assert l2w <= 1e-3, (name, l2w)
        assert l2n <= 1e-3, (name, l2n)
