"""Pins of the oracle's image loss and of its multi-view gradient sum: closed
forms, finite differences of the loss value itself, and finite differences of
the summed multi-view loss (the gradient of a sum of per-view losses whose
parameters are shared)."""
import numpy as np
import pytest

import oracle
from paper_2501_12369_amd import scenes


@pytest.mark.parametrize("kind", [oracle.LOSS_L1, oracle.LOSS_L2])
def test_loss_closed_forms(kind):
    I = np.full((3, 4, 5), 0.75)
    T = np.full((3, 4, 5), 0.25)
    L, g = oracle.image_loss(I, T, kind)
    assert L == pytest.approx(0.5 if kind == oracle.LOSS_L1 else 0.25, rel=1e-15)
    assert np.allclose(g, (1.0 if kind == oracle.LOSS_L1 else 1.0) / 60.0, rtol=1e-15)
    # sign flips with the difference; equal values give a zero gradient
    L0, g0 = oracle.image_loss(T, T, kind)
    assert L0 == 0.0 and np.all(g0 == 0.0)
    _, gneg = oracle.image_loss(T, I, kind)
    assert np.allclose(gneg, -g)


@pytest.mark.parametrize("kind", [oracle.LOSS_L1, oracle.LOSS_L2])
def test_loss_gradient_matches_finite_differences(kind):
    rng = np.random.default_rng(0)
    I = rng.uniform(0, 1, (3, 6, 7))
    T = rng.uniform(0, 1, (3, 6, 7))
    _, g = oracle.image_loss(I, T, kind)
    for idx in [(0, 0, 0), (1, 3, 4), (2, 5, 6)]:
        h = 1e-6
        Ip, Im = I.copy(), I.copy()
        Ip[idx] += h
        Im[idx] -= h
        fd = (oracle.image_loss(Ip, T, kind)[0] - oracle.image_loss(Im, T, kind)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-12)


def test_multiview_gradient_is_the_gradient_of_the_summed_loss(orc):
    sc = scenes.tiny(seed=1)
    sp = {k: v for k, v in sc["splats"].items()}
    cam0 = sc["camera"]
    cam1 = dict(cam0, width=48, height=40, cx=24.0, cy=20.0)
    cams = [oracle.camera_from_scene(c) for c in (cam0, cam1)]
    ko = oracle.KernelSpec(oracle.HALF_COS, 18.0 / np.pi, 1.36, 9.0)
    opts = oracle.make_opts()
    rng = np.random.default_rng(3)
    Gs = [rng.standard_normal((c.width * c.height, 3)) for c in cams]
    per_view, g3 = oracle.render_bwd_views(cams, ko, opts, sp, Gs)
    assert len(per_view) == 2

    def total(params):
        return sum(oracle.loss_linear(c, ko, opts, params, G) for c, G in zip(cams, Gs))

    checked = 0
    for name, idx in [("means", (0, 3)), ("means", (2, 10)), ("scales", (1, 5)), ("opacity", (7,)),
                      ("sh", (0, 1, 20))]:
        x = np.array(sp[name], dtype=np.float64)

        def f(xv, name=name):
            p = dict(sp)
            p[name] = xv
            return total(p)

        fd = oracle.fd_grad(f, x, idx)
        an = g3[name][idx]
        if abs(fd) < 1e-8 and abs(an) < 1e-8:
            continue
        assert an == pytest.approx(fd, rel=2e-4, abs=1e-7), (name, idx)
        checked += 1
    assert checked >= 3
