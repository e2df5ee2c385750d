"""Pins of the oracle's 1D signal-reconstruction experiment (no GPU): the
mixture against its closed form for one Gaussian component, the analytic
gradients against central differences of the loss, and convergence of the
Adam steps to an exactly representable target."""
import math

import numpy as np
import pytest

import oracle
from oracle import fit1d
from paper_2501_12369_amd import scenes

PI = math.pi
KINDS = {"G": (oracle.GAUSS, 2.0, 9.0, 0.0), "HC": (oracle.HALF_COS, 18 / PI, 9.0, 0.0),
         "RC": (oracle.RAISED_COS, 2.5 / PI, 6.25, 0.0), "Sinc": (oracle.SINC, 3 / PI, 9.0, 0.0),
         "RC_n2": (oracle.RAISED_COS_BETA, 2.5 / PI, 25.0, 1.0)}


def test_single_gaussian_component_closed_form(orc):
    x = np.linspace(-1, 1, 101)
    mu, sig, a = 0.1, 0.2, 0.7
    f, *_ = fit1d.mixture(oracle.GAUSS, 2.0, 9.0, 0.0, x, [[mu], [math.log(sig)], [a]])
    ref = a * np.exp(-((x - mu) / sig) ** 2 / 2.0)
    ref[((x - mu) / sig) ** 2 > 9.0] = 0.0
    assert np.allclose(f, ref, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("name", list(KINDS))
def test_gradients_match_central_differences(orc, name):
    kind, xi, e_max, beta = KINDS[name]
    x, sig = scenes.signals1d(257)
    t = sig["triangle"]
    p = scenes.fit1d_init(3, 6).astype(np.float64)
    p[2] = np.array([0.5, -0.2, 0.8, 0.3, 0.6, 0.4])
    L, g = fit1d.loss_and_grads(kind, xi, e_max, beta, x, t, p)
    checked = 0
    for row in range(3):
        for k in range(6):
            h = 1e-6
            pp, pm = p.copy(), p.copy()
            pp[row, k] += h
            pm[row, k] -= h
            fd = (fit1d.loss_and_grads(kind, xi, e_max, beta, x, t, pp)[0]
                  - fit1d.loss_and_grads(kind, xi, e_max, beta, x, t, pm)[0]) / (2 * h)
            # a sample crossing the support edge inside the stencil makes the difference one-sided
            _, _, _, Ep, _, _ = fit1d.mixture(kind, xi, e_max, beta, x, pp)
            _, _, _, Em, _, _ = fit1d.mixture(kind, xi, e_max, beta, x, pm)
            if not np.array_equal(Ep <= e_max, Em <= e_max):
                continue
            assert g[row, k] == pytest.approx(fd, rel=1e-5, abs=1e-8), (row, k)
            checked += 1
    assert checked >= 15


def test_adam_steps_recover_an_exact_mixture(orc):
    """A target that is itself a two-component half-cosine mixture is recovered
    by the Adam steps from a perturbed start (loss to ~0, parameters to the
    truth).  The half-cosine vanishes at its support edge, so the loss is
    smooth; the truncated Gaussian's jump of exp(-4.5) at E = 9 can stall it."""
    x = np.linspace(-1, 1, 201)
    truth = np.array([[-0.3, 0.35], [math.log(0.15), math.log(0.2)], [0.8, 0.5]])
    t, *_ = fit1d.mixture(oracle.HALF_COS, 18 / PI, 9.0, 0.0, x, truth)
    p0 = truth + np.array([[0.05, -0.04], [0.1, -0.1], [-0.1, 0.1]])
    z = np.zeros_like(p0)
    p, _, _, losses = fit1d.fit_steps(oracle.HALF_COS, 18 / PI, 9.0, 0.0, x, t, p0, z, z, 2000, 0,
                                      (3e-3, 3e-3, 3e-3))
    assert losses[-1] < 1e-20 < losses[0]
    assert np.allclose(p, truth, atol=1e-9)
