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


def psi_closed_form(kind: int, xi: float, e_max: float) -> float:
    """c_F of the kernel ``kind`` with scale ``xi`` restricted to E <= e_max."""
    rmax = math.sqrt(e_max) if math.isfinite(e_max) else math.inf

    def F(r):
        return float(kernel_value(kind, xi, r * r)[0])

    num, _ = integrate.quad(lambda r: r ** 4 * F(r), 0.0, rmax, limit=200, epsabs=0, epsrel=1e-12)
    den, _ = integrate.quad(lambda r: r ** 2 * F(r), 0.0, rmax, limit=200, epsabs=0, epsrel=1e-12)
    return num / (3.0 * den)


__all__ = ["psi_closed_form", "GAUSS", "HALF_COS", "RAISED_COS", "SINC", "IMQ", "IMQ_SQRT", "PARABOLA"]
