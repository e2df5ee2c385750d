"""Closed form of the correction factor psi (DARB Projection; Table 2).

TEST INFRASTRUCTURE ONLY (part of the oracle package).

The paper obtains psi by integrating a 3D DARBF along one axis (Simpson's rule,
Monte Carlo experiments section) and comparing the weighted covariance of the
resulting 2D density with the upper-left 2x2 block of the 3D covariance.

For a radial kernel K(x) = F(|x|^2) with identity covariance the marginal
density over (x, y) has covariance  c_F * I  with

    c_F = (1/3) * int r^4 F(r^2) dr / int r^2 F(r^2) dr      (r over the support),

because the second moment of an isotropic 3D density is split equally between
the three axes.  A linear change of variables x -> L x maps the kernel with
covariance parameter Sigma = L L^T to the general case, and marginalising
commutes with it, so the ratio is c_F for every Sigma: the scalar psi of the
paper is c_F of its kernel.
"""
from __future__ import annotations

import math

from scipy import integrate

from . import GAUSS, HALF_COS, IMQ, IMQ_SQRT, PARABOLA, RAISED_COS, SINC, kernel_value


def psi_closed_form(kind: int, xi: float, e_max: float, beta: float = 0.0) -> float:
    """c_F of the kernel ``kind`` with scale ``xi`` restricted to E <= e_max."""
    rmax = math.sqrt(e_max) if math.isfinite(e_max) else math.inf

    def F(r):
        return float(kernel_value(kind, xi, r * r, beta)[0])

    num, _ = integrate.quad(lambda r: r ** 4 * F(r), 0.0, rmax, limit=200, epsabs=0, epsrel=1e-12)
    den, _ = integrate.quad(lambda r: r ** 2 * F(r), 0.0, rmax, limit=200, epsabs=0, epsrel=1e-12)
    return num / (3.0 * den)


__all__ = ["psi_closed_form", "psi_grid_covariances", "psi_fit", "GAUSS", "HALF_COS", "RAISED_COS", "SINC", "IMQ", "IMQ_SQRT", "PARABOLA"]


# ---------------------------------------------------------------------------
# The paper's correction-factor experiment written out (Mathematical
# Expressions of Monte Carlo Experiments; the psi regression of the extended
# results), plain and slow: the kernel sampled on a 3D grid, summed along z
# with Simpson's rule, the weighted covariance of the 2D density, and the
# least-squares fits.  The grid holds the support's bounding box: half-extent
# (1 + 2/(n-1)) sqrt(e_max Sigma_aa) on axis a, n points per axis (n odd).
# ---------------------------------------------------------------------------

def psi_grid_covariances(kind: int, xi: float, e_max: float, sigma, n: int, beta: float = 0.0):
    """sigma [m, 6] = (xx, xy, xz, yy, yz, zz) -> [m, 3] = (a', b', d') of each 2D density."""
    import numpy as np
    from scipy.integrate import simpson

    from . import kernel_values

    sigma = np.asarray(sigma, np.float64)
    out = np.zeros((len(sigma), 3))
    margin = 1.0 + 2.0 / (n - 1)
    t = np.linspace(-1.0, 1.0, n)
    for s, (a, b, c, d, e, f) in enumerate(sigma):
        S = np.array([[a, b, c], [b, d, e], [c, e, f]])
        Sinv = np.linalg.inv(S)
        L = margin * np.sqrt(e_max * np.array([a, d, f]))
        gx, gy, gz = L[0] * t, L[1] * t, L[2] * t
        X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
        P = np.stack([X, Y, Z], -1)
        E = np.maximum(np.einsum("...i,ij,...j->...", P, Sinv, P), 0.0)
        dens = np.where(E <= e_max, kernel_values(kind, xi, np.minimum(E, e_max), beta), 0.0)
        w = simpson(dens, x=gz, axis=2)
        xx, yy = X[:, :, 0], Y[:, :, 0]
        W = w.sum()
        mx, my = (w * xx).sum() / W, (w * yy).sum() / W
        out[s] = [(w * (xx - mx) ** 2).sum() / W, (w * (xx - mx) * (yy - my)).sum() / W,
                  (w * (yy - my) ** 2).sum() / W]
    return out


def psi_fit(sigma, cov2):
    """Least squares without intercept: (a, b, c, d, e, f) -> (a', b', d') [3, 6],
    and the scalar psi minimising sum |Sigma'_2x2 - psi Sigma_2x2|_F^2."""
    import numpy as np

    X = np.asarray(sigma, np.float64)
    Y = np.asarray(cov2, np.float64)
    coef, *_ = np.linalg.lstsq(X, Y, rcond=None)
    num = np.sum(Y[:, 0] * X[:, 0] + 2 * Y[:, 1] * X[:, 1] + Y[:, 2] * X[:, 3])
    den = np.sum(X[:, 0] ** 2 + 2 * X[:, 1] ** 2 + X[:, 3] ** 2)
    return coef.T, float(num / den)
