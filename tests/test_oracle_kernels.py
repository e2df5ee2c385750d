"""Pins of the oracle's kernel profiles and correction factors against what the
paper prints and against closed forms (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import psi as psimod

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
PI = math.pi

# (kind, xi, e_max) with xi from Table 2 and the support of each kernel's listing
KERNELS = {
    "G": (oracle.GAUSS, 2.0, 9.0),
    "HC": (oracle.HALF_COS, 18.0 / PI, 9.0),
    "RC": (oracle.RAISED_COS, 2.5 / PI, 6.25),
    "Sinc": (oracle.SINC, 3.0 / PI, 9.0),
    "IMQ": (oracle.IMQ, 1.0, 9.0),
    "IMQ_SQRT": (oracle.IMQ_SQRT, 1.0, 9.0),
    "P": (oracle.PARABOLA, 9.0, 9.0),
}


def _xi_value(v):
    if isinstance(v, str):
        num, den = v.split("/")
        return float(num) / PI if den == "pi" else float(num) / float(den)
    return float(v)


@pytest.mark.parametrize("name", list(KERNELS))
def test_value_one_at_centre(orc, name):
    kind, xi, _ = KERNELS[name]
    assert orc.kernel_value(kind, xi, 0.0)[0] == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("name", ["HC", "RC", "Sinc", "P"])
def test_zero_at_support_limit(orc, name):
    # each single-pulse kernel reaches 0 exactly at the end of its main lobe
    kind, xi, e_max = KERNELS[name]
    assert abs(orc.kernel_value(kind, xi, e_max)[0]) < 1e-15


@pytest.mark.parametrize("name", list(KERNELS))
def test_decaying_on_support(orc, name):
    kind, xi, e_max = KERNELS[name]
    E = np.linspace(0.0, e_max, 401)
    F = orc.kernel_value(kind, xi, E)
    assert np.all(np.diff(F) < 0.0)
    assert np.all(F >= -1e-15)


def test_table2_xi_matches_oracle_constants():
    for name, v in GOLD["table2_xi"].items():
        if name.startswith("_"):
            continue
        assert _xi_value(v) == pytest.approx(KERNELS[name][1], rel=1e-15)


def test_hc_closed_values(orc):
    kind, xi, _ = KERNELS["HC"]
    # E = 4.5 -> cos(pi/4)
    assert orc.kernel_value(kind, xi, 4.5)[0] == pytest.approx(math.sqrt(0.5), abs=1e-15)
    # derivative closed form (half-cosine backward equations): -(1/xi) sin(E/xi)
    for E in (0.5, 3.0, 8.0):
        assert orc.kernel_deriv(kind, xi, E)[0] == pytest.approx(-(PI / 18) * math.sin(PI * E / 18), rel=1e-14)
    # extent matching: xi solves sqrt(2 pi xi lam) / 2 = 3 sqrt(lam)
    assert math.sqrt(2 * PI * xi) / 2 == pytest.approx(3.0, rel=1e-14)
    # the listings' constants approximate 1/xi = pi/18
    assert GOLD["hc_inverse_xi_listing"]["forward"] == pytest.approx(1 / xi, abs=6e-4)
    assert GOLD["hc_inverse_xi_listing"]["backward"] == pytest.approx(1 / xi, abs=6e-4)


def test_gauss_closed_value(orc):
    kind, xi, _ = KERNELS["G"]
    assert orc.kernel_value(kind, xi, 4.5)[0] == pytest.approx(math.exp(-2.25), rel=1e-15)
    assert orc.kernel_value(kind, xi, 9.0)[0] == pytest.approx(math.exp(-4.5), rel=1e-15)


def test_profile_plot_formulas(orc):
    # the kernel-comparison figure plots cos(2 pi x^2 / 36) and 1/sqrt(x^2 + 1) against x
    xs = np.array(GOLD["kernel_profile_plot"]["samples_x"])
    hc = orc.kernel_value(oracle.HALF_COS, 18.0 / PI, xs ** 2)
    assert np.allclose(hc, np.cos(2 * PI * xs ** 2 / 36.0), rtol=0, atol=1e-15)
    imq = orc.kernel_value(oracle.IMQ_SQRT, 1.0, xs ** 2)
    assert np.allclose(imq, 1.0 / np.sqrt(xs ** 2 + 1.0), rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", list(KERNELS))
def test_derivative_matches_central_difference(orc, name):
    kind, xi, e_max = KERNELS[name]
    for E in np.linspace(0.05, e_max - 0.05, 9):
        h = 1e-6
        fd = (orc.kernel_value(kind, xi, E + h)[0] - orc.kernel_value(kind, xi, E - h)[0]) / (2 * h)
        assert orc.kernel_deriv(kind, xi, E)[0] == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_derivative_limits_at_centre(orc):
    # raised cosine: d/dE [0.5 + 0.5 cos(sqrt(E)/xi)] -> -1/(4 xi^2); sinc: -> -1/(6 xi^2)
    _, xi, _ = KERNELS["RC"]
    assert orc.kernel_deriv(oracle.RAISED_COS, xi, 0.0)[0] == pytest.approx(-1 / (4 * xi * xi), rel=1e-12)
    _, xi, _ = KERNELS["Sinc"]
    assert orc.kernel_deriv(oracle.SINC, xi, 0.0)[0] == pytest.approx(-1 / (6 * xi * xi), rel=1e-12)
    # and the small-E branch joins the direct formula smoothly
    for E in (1e-7, 1e-5, 1e-3):
        u = math.sqrt(E) / xi
        direct = (u * math.cos(u) - math.sin(u)) / u ** 3 / (2 * xi * xi) if u > 1e-3 else None
        if direct is not None:
            assert orc.kernel_deriv(oracle.SINC, xi, E)[0] == pytest.approx(direct, rel=1e-6)


@pytest.mark.parametrize("name,printed", [("HC", 1.36), ("RC", 0.655), ("Sinc", 1.18), ("IMQ", 1.38), ("P", 1.3)])
def test_psi_closed_form_reproduces_listing_values(orc, name, printed):
    kind, xi, e_max = KERNELS[name]
    assert GOLD["listing_psi"][name] == printed
    assert psimod.psi_closed_form(kind, xi, e_max) == pytest.approx(printed, abs=0.015)


def test_psi_closed_form_table2():
    # Gaussian: untruncated marginal covariance ratio is exactly 1 (EWA closure)
    assert psimod.psi_closed_form(oracle.GAUSS, 2.0, math.inf) == pytest.approx(1.0, rel=1e-10)
    # IMQ of Table 1 (square-root form) gives Table 2's 1.61
    assert psimod.psi_closed_form(oracle.IMQ_SQRT, 1.0, 9.0) == pytest.approx(GOLD["table2_psi"]["IMQ"], abs=0.005)
    # RC, Sinc, P of Table 2 within rounding of the printed two digits
    for name in ("RC", "Sinc", "P"):
        kind, xi, e_max = KERNELS[name]
        assert psimod.psi_closed_form(kind, xi, e_max) == pytest.approx(GOLD["table2_psi"][name], abs=0.015)
    # HC: the closed form agrees with the listings and the regression (1.36), not Table 2's 1.34
    kind, xi, e_max = KERNELS["HC"]
    c = psimod.psi_closed_form(kind, xi, e_max)
    assert abs(c - GOLD["regression_hc_diagonal"]["a_prime_from_a"]) < 0.005
    assert abs(c - GOLD["table2_psi"]["HC"]) > 0.015


def test_psi_marginal_by_simpson_matches_closed_form(orc):
    """The paper's own experiment in miniature: sum a 3D half-cosine kernel along z
    on a grid (Simpson), take the weighted covariance of the 2D density, compare
    with the 2x2 block of the 3D covariance."""
    from scipy.integrate import simpson

    rng = np.random.default_rng(7)
    A = rng.standard_normal((3, 3))
    Sigma = A @ A.T + 0.5 * np.eye(3)
    Sinv = np.linalg.inv(Sigma)
    kind, xi, e_max = KERNELS["HC"]
    L = 3.2 * math.sqrt(np.max(np.linalg.eigvalsh(Sigma)))
    g = np.linspace(-L, L, 161)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    P = np.stack([X, Y, Z], -1)
    E = np.einsum("...i,ij,...j->...", P, Sinv, P)
    dens = np.where(E <= e_max, np.cos(np.minimum(E, e_max) / xi), 0.0)
    d2 = simpson(dens, x=g, axis=2)
    w = d2 / d2.sum()
    xx, yy = X[:, :, 0], Y[:, :, 0]
    mx, my = (w * xx).sum(), (w * yy).sum()
    cov = np.array([[(w * (xx - mx) ** 2).sum(), (w * (xx - mx) * (yy - my)).sum()],
                    [(w * (xx - mx) * (yy - my)).sum(), (w * (yy - my) ** 2).sum()]])
    ratio = cov / Sigma[:2, :2]
    c = psimod.psi_closed_form(kind, xi, e_max)
    assert np.allclose(ratio, c, rtol=0.01)


# ---------------------------------------------------------------- modified forms (Table 1, generic beta)

MODIFIED = {  # modified kind -> the fixed kind it reduces to, and that kind's beta
    oracle.GAUSS_BETA: (oracle.GAUSS, 2.0),
    oracle.HALF_COS_BETA: (oracle.HALF_COS, 2.0),
    oracle.RAISED_COS_BETA: (oracle.RAISED_COS, 1.0),
    oracle.SINC_BETA: (oracle.SINC, 1.0),
}


@pytest.mark.parametrize("mkind", list(MODIFIED))
def test_modified_forms_reduce_to_the_fixed_kernels(orc, mkind):
    """At the roll-off the listings use (beta = 2 for the Gaussian and the
    half-cosine, beta = 1 for the raised cosine and the sinc) the modified form
    of Table 1 is the fixed kernel: values and derivatives agree (two code paths:
    pow(E, beta/2) against the fixed forms in E or sqrt(E))."""
    kind, beta = MODIFIED[mkind]
    name = {oracle.GAUSS: "G", oracle.HALF_COS: "HC", oracle.RAISED_COS: "RC", oracle.SINC: "Sinc"}[kind]
    _, xi, e_max = KERNELS[name]
    E = np.concatenate([[0.0, 1e-9, 1e-4], np.linspace(0.01, e_max, 57)])
    assert np.allclose(orc.kernel_value(mkind, xi, E, beta), orc.kernel_value(kind, xi, E), rtol=1e-13, atol=1e-15)
    Ed = E[1:]
    assert np.allclose(orc.kernel_deriv(mkind, xi, Ed, beta), orc.kernel_deriv(kind, xi, Ed), rtol=1e-9, atol=1e-12)


def test_modified_closed_values(orc):
    # modified Gaussian, beta = 4, xi = 2: exp(-d_M^4 / 2)
    assert orc.kernel_value(oracle.GAUSS_BETA, 2.0, 1.0, 4.0)[0] == pytest.approx(math.exp(-0.5), rel=1e-14)
    assert orc.kernel_value(oracle.GAUSS_BETA, 2.0, 4.0, 4.0)[0] == pytest.approx(math.exp(-8.0), rel=1e-14)
    # modified half-cosine, beta = 1: zero at the end of the main lobe d_M / xi = pi / 2
    xi = 2.0
    assert orc.kernel_value(oracle.HALF_COS_BETA, xi, (xi * PI / 2) ** 2, 1.0)[0] == pytest.approx(0.0, abs=1e-15)
    assert orc.kernel_value(oracle.HALF_COS_BETA, xi, (xi * PI / 3) ** 2, 1.0)[0] == pytest.approx(0.5, rel=1e-14)
    # raised cosine with n pulses (u <= n pi): 0 at the end of odd pulses, 1 at the end of even ones
    xi = 2.5 / PI
    for npulse, val in ((1, 0.0), (2, 1.0), (3, 0.0)):
        E = (xi * npulse * PI) ** 2
        assert orc.kernel_value(oracle.RAISED_COS_BETA, xi, E, 1.0)[0] == pytest.approx(val, abs=1e-14)
    # modular sinc with n pulses (u <= (n + 1) pi / 2): |sin u| / u
    xi = 3.0 / PI
    assert orc.kernel_value(oracle.SINC_BETA, xi, (xi * PI) ** 2, 1.0)[0] == pytest.approx(0.0, abs=1e-15)
    assert orc.kernel_value(oracle.SINC_BETA, xi, (xi * 1.5 * PI) ** 2, 1.0)[0] == pytest.approx(2 / (3 * PI),
                                                                                                  rel=1e-13)
    # a generic beta moves the lobe: beta = 3, half-cosine: cos(d_M^3 / xi)
    assert orc.kernel_value(oracle.HALF_COS_BETA, 4.0, 2.0 ** 2, 3.0)[0] == pytest.approx(math.cos(2.0), rel=1e-14)


@pytest.mark.parametrize("mkind", list(MODIFIED))
@pytest.mark.parametrize("beta", [1.0, 1.5, 3.0, 4.0])
def test_modified_derivative_matches_central_difference(orc, mkind, beta):
    xi = 1.3
    E = np.linspace(0.05, 8.0, 41)
    an = orc.kernel_deriv(mkind, xi, E, beta)
    h = 1e-6
    fd = (orc.kernel_value(mkind, xi, E + h, beta) - orc.kernel_value(mkind, xi, E - h, beta)) / (2 * h)
    assert np.allclose(an, fd, rtol=1e-6, atol=1e-9)


def test_modified_derivative_at_centre(orc):
    # beta = 2: dF/dE(0) = F'(0) / xi; beta > 2: 0; beta < 2: taken as 0 (every gradient it feeds vanishes)
    assert orc.kernel_deriv(oracle.GAUSS_BETA, 2.0, 0.0, 2.0)[0] == pytest.approx(-0.5, rel=1e-15)
    assert orc.kernel_deriv(oracle.GAUSS_BETA, 2.0, 0.0, 4.0)[0] == 0.0
    assert orc.kernel_deriv(oracle.HALF_COS_BETA, 2.0, 0.0, 1.0)[0] == 0.0
    assert orc.kernel_deriv(oracle.SINC_BETA, 1.0, 0.0, 1.0)[0] == 0.0
    # beta = 1 near the centre: dF/dE ~ F'(u) / (2 xi sqrt(E)) -- finite for E > 0
    E = 1e-10
    d = orc.kernel_deriv(oracle.GAUSS_BETA, 2.0, E, 1.0)[0]
    assert d == pytest.approx(-1.0 / (2 * 2.0 * math.sqrt(E)), rel=1e-4)
