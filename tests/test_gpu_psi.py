"""The correction-factor experiment on the GPU (darb_psi_calibrate through the
C ABI) against the oracle's plain grid experiment on the same covariances and
grid: every sample's 2D covariance (a', b', d') within 1e-5 of its scale (the
GPU evaluates E and F in FP32 and sums in FP64), the fitted map and the scalar
psi within 1e-5; and, on a finer grid, psi against the closed form c_F."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import psi as psimod
from paper_2501_12369_amd import calibrate, native, pipeline, scenes

from gpu_util import ORACLE_KERNELS

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kname", list(ORACLE_KERNELS))
def test_psi_grid_matches_oracle(kname):
    print(f"psi calibration {kname}", flush=True)
    ko = ORACLE_KERNELS[kname]
    k = pipeline.KERNELS[kname]
    f32 = lambda v: float(np.float32(v))
    sig = scenes.covariances(21, 9)
    n = 33
    r = calibrate.calibrate_psi(k, sigma=sig, grid_n=n)
    cov_o = psimod.psi_grid_covariances(ko.kind, f32(ko.xi), f32(ko.e_max), sig, n, f32(ko.beta))
    scale = np.abs(sig[:, [0, 1, 3]]).max(1, keepdims=True)
    err = np.abs(r["cov2"] - cov_o) / scale
    print(f"  worst cov err {err.max():.2e}")
    assert np.all(err <= 1e-5)
    coef_o, psi_o = psimod.psi_fit(sig, cov_o)
    assert np.allclose(r["coef"], coef_o, atol=1e-4)
    assert r["psi"] == pytest.approx(psi_o, rel=1e-5)


@pytest.mark.parametrize("kname", ["half_cos", "raised_cos", "parabola"])
def test_psi_fine_grid_matches_closed_form(kname):
    ko = ORACLE_KERNELS[kname]
    r = calibrate.calibrate_psi(pipeline.KERNELS[kname], m=200, grid_n=129, seed=3)
    c = psimod.psi_closed_form(ko.kind, ko.xi, ko.e_max, ko.beta)
    print(f"  {kname}: grid psi {r['psi']:.5f}, closed form {c:.5f}")
    assert r["psi"] == pytest.approx(c, rel=1e-3)


def test_psi_arguments():
    k = pipeline.KERNELS["half_cos"]
    sig = torch.zeros((4, 6), dtype=torch.float64, device="cuda")
    ws = torch.empty(native.darb_psi_calibrate_workspace(4, 33), dtype=torch.uint8, device="cuda")
    cov2 = torch.empty((4, 3), dtype=torch.float64, device="cuda")
    fit = torch.empty(19, dtype=torch.float64, device="cuda")
    for bad_n in (32, 3, 4097):
        with pytest.raises(native.DarbError):
            native.darb_psi_calibrate(k, 4, sig, bad_n, ws, cov2)
    with pytest.raises(native.DarbError):
        native.darb_psi_calibrate(k, 4, sig, 33, ws, cov2, fit)  # the fit needs >= 6 samples
