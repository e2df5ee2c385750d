"""The training-step companions on the GPU (through the C ABI) against the
oracle: L1 + D-SSIM loss value and gradient, one Adam step over several
parameter groups, the densification statistics; and a short optimisation on
the tiny scene whose loss goes down."""
import numpy as np
import pytest
import torch

import oracle
from paper_2501_12369_amd import native, pipeline, scenes

from gpu_util import dev, oracle_kernel_fp32, oracle_opts_fp32, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("W,H,lam", [(77, 61, 0.2), (1297, 840, 0.2), (40, 33, 1.0)])
def test_ssim_loss_matches_oracle(W, H, lam):
    print(f"ssim loss {W}x{H} lambda={lam}", flush=True)
    rng = np.random.default_rng(W)
    img = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    tgt = np.clip(img + rng.normal(0, 0.1, img.shape), 0, 1).astype(np.float32)
    ws = torch.empty(native.darb_ssim_loss_workspace(W, H), dtype=torch.uint8, device="cuda")
    dL = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    Ld = torch.empty(4, dtype=torch.float32, device="cuda")
    native.darb_ssim_loss(dev(img), dev(tgt), W, H, lam, dL, loss_dev=Ld, ws=ws)
    L1 = float(Ld[0])
    native.darb_ssim_loss(dev(img), dev(tgt), W, H, lam, dL, loss_dev=Ld, ws=ws)
    torch.cuda.synchronize()
    assert float(Ld[0]) == L1  # fixed summation order
    Lo, go = oracle.ssim_loss(img, tgt, lam)
    print(f"  loss gpu {L1:.7f} oracle {Lo:.7f}")
    assert L1 == pytest.approx(Lo, rel=1e-5)
    g = to_np(dL)
    keep = np.abs(img.astype(np.float64) - tgt) > 1e-5  # the L1 sign is a decision
    rel = np.linalg.norm((g - go)[keep]) / np.linalg.norm(go[keep])
    print(f"  grad relL2 {rel:.2e}")
    assert rel <= 1e-4
    assert np.all(np.abs(g - go)[keep] <= 1e-3 * np.abs(go[keep]) + 1e-4 * np.abs(go).max())


def test_adam_matches_oracle():
    rng = np.random.default_rng(5)
    sizes, lrs = (1000, 777, 3), (1e-3, 5e-2, 1.0)
    P = [rng.standard_normal(s).astype(np.float32) for s in sizes]
    groups = [dict(param=dev(p), grad=torch.empty(s, device="cuda"), m=torch.zeros(s, device="cuda"),
                   v=torch.zeros(s, device="cuda"), lr=lr) for p, s, lr in zip(P, sizes, lrs)]
    ref = [(p.astype(np.float64), np.zeros(s), np.zeros(s)) for p, s in zip(P, sizes)]
    for step in range(1, 4):
        G = [rng.standard_normal(s).astype(np.float32) for s in sizes]
        for g, gg in zip(groups, G):
            g["grad"].copy_(torch.from_numpy(gg))
        native.darb_adam(groups, step, 0.9, 0.999, 1e-15)
        # the oracle receives the hyper-parameters as the GPU does (FP32)
        f = lambda x: float(np.float32(x))
        ref = [oracle.adam_step(p, gg, m, v, step, f(lr), beta1=f(0.9), beta2=f(0.999), eps=f(1e-15))
               for (p, m, v), gg, lr in zip(ref, G, lrs)]
    torch.cuda.synchronize()
    for g, (p, m, v) in zip(groups, ref):
        assert np.allclose(to_np(g["param"]), p, rtol=1e-5, atol=1e-6)
        assert np.allclose(to_np(g["m"]), m, rtol=1e-5, atol=1e-7)
        assert np.allclose(to_np(g["v"]), v, rtol=1e-5, atol=1e-9)


def test_densify_stats_match_oracle():
    rng = np.random.default_rng(6)
    n = 10000
    gxy = rng.standard_normal((n, 2)).astype(np.float32)
    r = rng.integers(-1, 6, n).astype(np.int32)
    acc0 = rng.uniform(0, 1, n).astype(np.float32)
    cnt0 = rng.integers(0, 5, n).astype(np.int32)
    mr0 = rng.integers(0, 8, n).astype(np.int32)
    g2d = dict(xy=dev(gxy), conic=torch.zeros((n, 3), device="cuda"), opacity=torch.zeros(n, device="cuda"),
               rgb=torch.zeros((n, 3), device="cuda"))
    acc, cnt, mr = dev(acc0), dev(cnt0), dev(mr0)
    native.darb_densify_stats(g2d, dev(r), n, acc, cnt, mr)
    torch.cuda.synchronize()
    a, c, m = oracle.densify_stats(gxy, r, acc0, cnt0, mr0)
    assert np.allclose(to_np(acc), a, rtol=1e-6)
    assert np.array_equal(to_np(cnt), c) and np.array_equal(to_np(mr), m)


def test_short_optimisation_reduces_the_loss():
    print("tiny scene: 40 Adam steps on L1 + D-SSIM", flush=True)
    sc = scenes.tiny(seed=1)
    sp, cam = sc["splats"], sc["camera"]
    n, W, H = sp["means"].shape[1], cam["width"], cam["height"]
    kern = pipeline.KERNELS["half_cos"]
    # target: the oracle's render of the scene; start: perturbed means and colours
    _, img = oracle.render(oracle.camera_from_scene(cam), oracle_kernel_fp32("half_cos"), oracle_opts_fp32(),
                           {k: v for k, v in sp.items()})
    target = dev(img["rgb"].T.reshape(3, H, W).astype(np.float32))
    rng = np.random.default_rng(7)
    start = dict(sp)
    start["means"] = (sp["means"] + rng.normal(0, 0.05, sp["means"].shape)).astype(np.float32)
    start["sh"] = (sp["sh"] + rng.normal(0, 0.2, sp["sh"].shape)).astype(np.float32)
    spd = pipeline.splats_to_device(start)
    names = ("means", "scales", "quats", "opacity", "sh")
    lrs = dict(means=2e-3, scales=1e-3, quats=1e-3, opacity=1e-3, sh=1e-2)
    g2d, g3d = pipeline.alloc_grads(n, int(spd["sh_degree"]))
    state = {k: (torch.zeros_like(spd[k]), torch.zeros_like(spd[k])) for k in names}
    ws = torch.empty(native.darb_ssim_loss_workspace(W, H), dtype=torch.uint8, device="cuda")
    dL = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    Ld = torch.empty(4, dtype=torch.float32, device="cuda")
    losses = []
    for step in range(1, 41):
        fr = pipeline.render(spd, cam, kern)
        native.darb_ssim_loss(fr.image, target, W, H, 0.2, dL, loss_dev=Ld, ws=ws)
        pipeline.render_backward(fr, dL, spd, cam, kern, grads=(g2d, g3d))
        native.darb_adam([dict(param=spd[k], grad=g3d[k], m=state[k][0], v=state[k][1], lr=lrs[k]) for k in names],
                         step)
        losses.append(float(Ld[0]))
    print(f"  loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    assert losses[-1] < 0.7 * losses[0]
