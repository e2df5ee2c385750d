"""Pins of the oracle's training-step companions: the window filter against
scipy's 1D convolution with zero padding, SSIM closed forms (identical images,
constant images in the interior), finite differences of the L1 + D-SSIM loss,
Adam against torch.optim.Adam, and the densification statistics by hand."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

import oracle


def test_window_filter_matches_scipy():
    rng = np.random.default_rng(0)
    a = rng.uniform(0, 1, (23, 31))
    g = oracle.ssim_window()
    assert g.sum() == pytest.approx(1.0, abs=1e-15) and np.allclose(g, g[::-1])
    ref = ndi.convolve1d(ndi.convolve1d(a, g, axis=1, mode="constant"), g, axis=0, mode="constant")
    assert np.allclose(oracle.window_filter(a), ref, rtol=0, atol=1e-14)


def test_ssim_closed_forms():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (20, 24))
    S, *_ = oracle.ssim_map(x, x)
    assert np.allclose(S, 1.0, atol=1e-12)
    a, b = 0.7, 0.2
    S, *_ = oracle.ssim_map(np.full((30, 30), a), np.full((30, 30), b))
    interior = S[5:-5, 5:-5]  # full window inside: zero variance, means a and b
    expect = (2 * a * b + oracle.SSIM_C1) / (a * a + b * b + oracle.SSIM_C1)
    assert np.allclose(interior, expect, rtol=1e-12)
    # identical images: loss is the L1 weight times zero, gradient of the SSIM term vanishes
    L, g = oracle.ssim_loss(np.stack([x] * 3), np.stack([x] * 3), 0.2)
    assert abs(L) < 1e-12 and np.abs(g).max() < 1e-12


@pytest.mark.parametrize("lam", [0.0, 0.2, 1.0])
def test_ssim_loss_gradient_matches_finite_differences(lam):
    rng = np.random.default_rng(2)
    I = rng.uniform(0, 1, (3, 14, 17))
    T = rng.uniform(0, 1, (3, 14, 17))
    _, g = oracle.ssim_loss(I, T, lam)
    for idx in [(0, 0, 0), (1, 7, 8), (2, 13, 16), (0, 3, 12), (2, 10, 1)]:
        h = 1e-6
        Ip, Im = I.copy(), I.copy()
        Ip[idx] += h
        Im[idx] -= h
        fd = (oracle.ssim_loss(Ip, T, lam)[0] - oracle.ssim_loss(Im, T, lam)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-5, abs=1e-10)


def test_adam_matches_torch():
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(4)]
    t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step, g in enumerate(grads, start=1):
        t.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = oracle.adam_step(p, g, m, v, step, 1e-2)
    assert np.allclose(p, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_densify_stats_by_hand():
    g = np.array([[3.0, 4.0], [1.0, 0.0], [0.0, 2.0]])
    r = np.array([2, 0, 5])
    acc, cnt, mr = oracle.densify_stats(g, r, np.array([1.0, 1.0, 0.0]), np.array([1, 0, 2]), np.array([3, 9, 4]))
    assert np.allclose(acc, [6.0, 1.0, 2.0]) and list(cnt) == [2, 0, 3] and list(mr) == [3, 9, 5]
