"""Pins of the oracle's correction-factor experiment (the grid marginal with
Simpson's rule along z, its weighted covariance, the least-squares fits)
against the closed form c_F of each kernel (a different method: 1D quadrature
of the radial moments) and the values the paper prints (Table 2, the
half-cosine regression of the extended results).  No GPU."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import psi as psimod
from paper_2501_12369_amd import scenes

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
PI = math.pi
N = 49  # grid points per axis


@pytest.fixture(scope="module")
def sig():
    return scenes.covariances(5, 12)


@pytest.mark.parametrize("kind,xi,e_max,beta", [
    (oracle.GAUSS, 2.0, 9.0, 0.0), (oracle.HALF_COS, 18 / PI, 9.0, 0.0), (oracle.RAISED_COS, 2.5 / PI, 6.25, 0.0),
    (oracle.PARABOLA, 9.0, 9.0, 0.0), (oracle.HALF_COS_BETA, 6 / PI, 9.0, 1.0),
    (oracle.RAISED_COS_BETA, 2.5 / PI, 25.0, 1.0)])
def test_grid_marginal_covariance_is_c_F_times_the_block(orc, sig, kind, xi, e_max, beta):
    """Marginalising an elliptical kernel along z scales the 2x2 block by c_F
    for every covariance; the grid experiment reproduces it within its
    discretisation error."""
    c = psimod.psi_closed_form(kind, xi, e_max, beta)
    cov2 = psimod.psi_grid_covariances(kind, xi, e_max, sig, N, beta)
    block = sig[:, [0, 1, 3]]
    scale = np.abs(block).max(1, keepdims=True)
    assert np.all(np.abs(cov2 - c * block) <= 4e-3 * c * scale)
    coef, psi = psimod.psi_fit(sig, cov2)
    assert psi == pytest.approx(c, rel=2e-3)


def test_half_cosine_regression_matches_the_printed_one(orc):
    """The printed regression for the half-cosine: 1.36 on a -> a', b -> b',
    d -> d'.  The fitted off-diagonal weights vanish (an elliptical kernel's
    marginal depends on the 2x2 block only); the printed ones (-0.2 b, -0.1 c in
    a', -0.2 c and 0.1 e in d') are read as noise of a fit to sampled data."""
    sig = scenes.covariances(6, 40)
    cov2 = psimod.psi_grid_covariances(oracle.HALF_COS, 18 / PI, 9.0, sig, 41)
    coef, psi = psimod.psi_fit(sig, cov2)
    g = GOLD["regression_hc_diagonal"]
    assert coef[0, 0] == pytest.approx(g["a_prime_from_a"], abs=0.01)
    assert coef[1, 1] == pytest.approx(g["b_prime_from_b"], abs=0.01)
    assert coef[2, 3] == pytest.approx(g["d_prime_from_d"], abs=0.01)
    off = coef.copy()
    off[0, 0] = off[1, 1] = off[2, 3] = 0.0
    assert np.abs(off).max() < 0.02
    assert psi == pytest.approx(GOLD["listing_psi"]["HC"], abs=0.01)


@pytest.mark.parametrize("name,kind,xi,e_max", [("RC", oracle.RAISED_COS, 2.5 / PI, 6.25),
                                                ("Sinc", oracle.SINC, 3 / PI, 9.0),
                                                ("P", oracle.PARABOLA, 9.0, 9.0),
                                                ("IMQ", oracle.IMQ_SQRT, 1.0, 9.0)])
def test_grid_psi_reproduces_table2(orc, name, kind, xi, e_max):
    sig = scenes.covariances(7, 8)
    _, psi = psimod.psi_fit(sig, psimod.psi_grid_covariances(kind, xi, e_max, sig, 41))
    assert psi == pytest.approx(GOLD["table2_psi"][name], abs=0.015)


def test_gaussian_untruncated_limit(orc):
    # with the support far out the Gaussian's marginal keeps the block (EWA closure): psi -> 1
    sig = scenes.covariances(8, 6)
    cov2 = psimod.psi_grid_covariances(oracle.GAUSS, 2.0, 64.0, sig, 61)
    assert np.allclose(cov2, sig[:, [0, 1, 3]], rtol=2e-3, atol=2e-3 * np.abs(sig).max())
