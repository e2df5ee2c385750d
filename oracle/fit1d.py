"""The 1D signal-reconstruction experiment, plain FP64 (Assessing DARBFs through
1D Simulations; the extended 1D results).

TEST INFRASTRUCTURE ONLY (part of the oracle package).

A target t sampled at points x is approximated by a mixture of DARBF
components, f(x) = sum_k a_k F(E_k(x)) with E_k(x) = ((x - mu_k) / sigma_k)^2
(the squared Mahalanobis distance in one dimension), each term zero where
E_k > e_max; the loss is the mean squared error, and Adam updates
(mu_k, log sigma_k, a_k).  Written out step by step in the order the
experiment takes them: forward, residual, loss, gradients, Adam.
"""
from __future__ import annotations

import numpy as np

from . import adam_step, kernel_derivs, kernel_values


def mixture(kind, xi, e_max, beta, x, params):
    """f(x) and the per-component terms' ingredients (E, inside, F, dF/dE)."""
    mu, ls, a = (np.asarray(p, np.float64) for p in params)
    x = np.asarray(x, np.float64)
    d = x[:, None] - mu[None, :]
    sig = np.exp(ls)
    E = (d / sig[None, :]) ** 2
    inside = E <= e_max
    F = np.where(inside, kernel_values(kind, xi, np.minimum(E, e_max), beta), 0.0)
    dF = np.where(inside, kernel_derivs(kind, xi, np.minimum(E, e_max), beta), 0.0)
    return F @ a, d, sig, E, F, dF


def loss_and_grads(kind, xi, e_max, beta, x, t, params):
    """L = mean (f - t)^2 and dL/d(mu, log sigma, a), each [n]."""
    mu, ls, a = (np.asarray(p, np.float64) for p in params)
    f, d, sig, E, F, dF = mixture(kind, xi, e_max, beta, x, params)
    r = f - np.asarray(t, np.float64)
    m = len(r)
    L = float(np.mean(r * r))
    g_a = 2.0 / m * (r @ F)
    common = 2.0 / m * (r[:, None] * a[None, :] * dF)  # dL/dE_k at each sample
    g_mu = np.sum(common * (-2.0 * d / sig[None, :] ** 2), axis=0)  # dE/dmu = -2 (x - mu) / sigma^2
    g_ls = np.sum(common * (-2.0 * E), axis=0)                      # dE/dlog sigma = -2 E
    return L, np.stack([g_mu, g_ls, g_a])


def fit_steps(kind, xi, e_max, beta, x, t, params, m1, m2, steps, step0, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """``steps`` Adam steps; returns (params [3, n], m1, m2, losses [steps])."""
    p = np.array(params, np.float64)
    m1 = np.array(m1, np.float64)
    m2 = np.array(m2, np.float64)
    losses = []
    for s in range(steps):
        L, g = loss_and_grads(kind, xi, e_max, beta, x, t, p)
        losses.append(L)
        for row in range(3):
            p[row], m1[row], m2[row] = adam_step(p[row], g[row], m1[row], m2[row], step0 + s + 1, lr[row], beta1,
                                                 beta2, eps)
    return p, m1, m2, np.array(losses)
