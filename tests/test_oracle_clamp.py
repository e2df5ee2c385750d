"""Pins of the oracle's Jacobian clamp (DARB Projection: the affine Jacobian J
of the perspective map in the 2x2 covariance projection; the clamp of
|t_x/t_z|, |t_y/t_z| to jac_clamp times the half field of view is the 3DGS
pipeline's, which the paper keeps).  No GPU.

Forward: for a splat whose centre lies beyond the limit, the oracle's 2D
covariance must equal psi * A Sigma A^T + eps I with A the derivative of the
pinhole map taken by central differences at the *boundary* point (t_z times the
clamped ratios, same depth), Sigma built from scipy's rotation; the projected
mean must stay the unclamped pinhole image of the centre.  A clamp applied to
the wrong coordinate, with the wrong sign on the negative side, with width and
height swapped, or leaking into the mean fails here (W != H, fx != fy).

Backward: central differences of the oracle's full forward (preprocess +
composite) over splats beyond the limit in +x, -x, +y, -y and a corner; they
match the analytic backward only if the gradient through J vanishes across an
active clamp (the mean still moves the footprint's centre).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle

W, H = 96, 64
FX, FY, CX, CY = 80.0, 90.0, 48.0, 32.0
CLAMP = 1.3
LX, LY = CLAMP * 0.5 * W / FX, CLAMP * 0.5 * H / FY  # 0.78, 0.4622
HC = oracle.KernelSpec(oracle.HALF_COS, 18.0 / math.pi, 1.36, 9.0)
GA = oracle.KernelSpec(oracle.GAUSS, 2.0, 1.0, 9.0)


def _cam(orc, jac_clamp=CLAMP, dilation=0.3):
    # world frame = camera frame (identity view), camera at the origin
    return orc.make_camera(np.eye(4), np.zeros(3), FX, FY, CX, CY, W, H, near_z=0.2, jac_clamp=jac_clamp,
                           dilation=dilation)


def _pinhole(t):
    return np.array([FX * t[0] / t[2] + CX, FY * t[1] / t[2] + CY])


def _jacobian_fd(t):
    A = np.zeros((2, 3))
    for c in range(3):
        e = np.zeros(3)
        e[c] = 1e-6 * max(1.0, abs(t[c]))
        A[:, c] = (_pinhole(t + e) - _pinhole(t - e)) / (2 * e[c])
    return A


def _params(mus, scales, quats, opacity=0.7, colours=None):
    n = len(mus)
    rng = np.random.default_rng(3)
    rgb = rng.uniform(0.2, 0.9, (n, 3)) if colours is None else np.asarray(colours)
    sh = ((rgb - 0.5) / 0.28209479177387814).T.reshape(1, 3, n)
    return dict(means=np.asarray(mus, float).T.copy(), scales=np.asarray(scales, float).T.copy(),
                quats=np.asarray(quats, float).T.copy(), opacity=np.full(n, opacity), sh=sh, sh_degree=0)


# ratios t/t_z of centres: beyond the limit in each direction, a corner, and inside
CASES = [(1.15 * LX, 0.1), (-1.2 * LX, -0.05), (0.2, 1.3 * LY), (-0.1, -1.25 * LY), (1.1 * LX, -1.1 * LY),
         (0.5 * LX, 0.5 * LY)]


@pytest.mark.parametrize("psi,eps", [(1.0, 0.0), (1.36, 0.3)])
@pytest.mark.parametrize("ratio", CASES)
def test_clamped_projection_uses_jacobian_at_the_boundary(orc, ratio, psi, eps):
    rx, ry = ratio
    z = 3.0
    mu = np.array([rx * z, ry * z, z])
    scale = np.array([0.9, 0.35, 0.6])
    q = np.array([0.8, 0.3, -0.4, 0.33])
    k = orc.KernelSpec(oracle.HALF_COS, 18.0 / math.pi, psi, 9.0)
    p = _params([mu], [scale], [q])
    proj = orc.preprocess(_cam(orc, dilation=eps), k, p["means"], p["scales"], p["quats"], p["sh"], 0)
    # expected, from definitions written independently of the oracle
    tb = np.array([np.clip(rx, -LX, LX) * z, np.clip(ry, -LY, LY) * z, z])
    A = _jacobian_fd(tb)
    Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scipy takes (x, y, z, w)
    Sigma = Rm @ np.diag(scale ** 2) @ Rm.T
    cov = psi * A @ Sigma @ A.T + eps * np.eye(2)
    got = proj["cov2d"][0]
    assert np.allclose(got, [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-7, atol=1e-9 * np.abs(cov).max())
    # the mean is the unclamped image of the centre
    assert proj["visible"][0] == 1
    assert np.allclose(proj["xy"][0], _pinhole(mu), rtol=1e-13)
    # beyond the limit the covariance no longer depends on the centre's ratio
    if abs(rx) > LX or abs(ry) > LY:
        mu2 = mu + np.array([0.3 * np.sign(rx) * (abs(rx) > LX), 0.2 * np.sign(ry) * (abs(ry) > LY), 0.0])
        p2 = _params([mu2], [scale], [q])
        proj2 = orc.preprocess(_cam(orc, dilation=eps), k, p2["means"], p2["scales"], p2["quats"], p2["sh"], 0)
        assert np.array_equal(proj2["cov2d"][0], got)


def test_clamp_disabled_is_plain_pinhole_jacobian(orc):
    # jac_clamp <= 0: J at the centre itself even far beyond the field of view
    z = 2.5
    mu = np.array([1.4 * LX * z, -1.3 * LY * z, z])
    scale, q = np.array([0.5, 0.2, 0.3]), np.array([0.2, 0.9, 0.1, -0.3])
    p = _params([mu], [scale], [q])
    proj = orc.preprocess(_cam(orc, jac_clamp=0.0, dilation=0.0), GA, p["means"], p["scales"], p["quats"], p["sh"], 0)
    A = _jacobian_fd(mu)
    Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    cov = A @ Rm @ np.diag(scale ** 2) @ Rm.T @ A.T
    assert np.allclose(proj["cov2d"][0], [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-7)


def _decisions(out):
    return out["last"].copy(), out["ncontrib"].copy()


@pytest.mark.parametrize("k", [HC, GA], ids=["HC", "G"])
def test_backward_through_active_clamp_matches_fd(orc, k):
    z = 3.0
    mus, scales, quats = [], [], []
    rng = np.random.default_rng(11)
    # centres beyond the limit whose footprints still reach into the image
    for rx, ry in CASES[:5]:
        mus.append([rx * z, ry * z, z + rng.uniform(-0.3, 0.3)])
        scales.append(rng.uniform(0.45, 0.8, 3))
        q = rng.standard_normal(4)
        quats.append(q / np.linalg.norm(q))
    p = _params(mus, scales, quats, opacity=0.6)
    cam = _cam(orc)
    opts = orc.make_opts()
    G = np.random.default_rng(12).standard_normal((W * H, 3))
    proj, g2d, g3d = orc.render_bwd(cam, k, opts, p, G)
    assert np.all(proj["visible"] == 1)
    tx = p["means"][0] / p["means"][2]
    ty = p["means"][1] / p["means"][2]
    assert np.sum((np.abs(tx) > LX) | (np.abs(ty) > LY)) == 5
    _, ref = orc.render(cam, k, opts, p)
    assert np.all(ref["ncontrib"] <= 5) and ref["ncontrib"].max() >= 1
    ref_d = _decisions(ref)

    def loss_at(name, index, val):
        pp = {kk: (v.copy() if isinstance(v, np.ndarray) else v) for kk, v in p.items()}
        pp[name][index] = val
        _, out = orc.render(cam, k, opts, pp)
        return float(np.sum(G * out["rgb"])), _decisions(out)

    checked = 0
    for name, ncomp in (("means", 3), ("scales", 3), ("quats", 4)):
        grad = g3d[name]
        scale = np.max(np.abs(grad))
        for i in range(5):
            for comp in range(ncomp):
                index = (comp, i)
                x0 = p[name][index]
                h = 1e-6 * max(1.0, abs(x0))
                fp, dp = loss_at(name, index, x0 + h)
                fm, dm = loss_at(name, index, x0 - h)
                if not all(np.array_equal(a, b) for a, b in zip(dp + dm, ref_d + ref_d)):
                    continue
                fd = (fp - fm) / (2 * h)
                assert abs(grad[index] - fd) <= 1e-5 * abs(fd) + 1e-7 * scale, (name, index, grad[index], fd)
                checked += 1
    assert checked >= 45
