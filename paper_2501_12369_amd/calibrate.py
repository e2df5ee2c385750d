"""The correction-factor experiment on the GPU (Mathematical Expressions of
Monte Carlo Experiments; the psi regression of the extended results): random
3D covariances, each kernel sampled on a grid over its support, summed along
one axis with Simpson's rule, the weighted covariance of the 2D density, and
the least-squares fits -- all in libdarb (darb_psi_calibrate); this module only
draws the covariances and moves the buffers.

    python -m paper_2501_12369_amd.calibrate [--m 1000] [--grid 97]

prints psi and the fitted 3 x 6 map for every preset kernel."""
from __future__ import annotations

import argparse

import numpy as np
import torch

from . import native, pipeline, scenes


def calibrate_psi(kernel, sigma: np.ndarray | None = None, m: int = 1000, grid_n: int = 97, seed: int = 0):
    """Returns dict(cov2 [m, 3] (a', b', d'), coef [3, 6], psi) for ``kernel``
    (a pipeline.KernelSpec; its psi is not used)."""
    if sigma is None:
        sigma = scenes.covariances(seed, m)
    m = len(sigma)
    sig = torch.as_tensor(np.ascontiguousarray(sigma, np.float64)).cuda()
    ws = torch.empty(max(native.darb_psi_calibrate_workspace(m, grid_n), 1), dtype=torch.uint8, device="cuda")
    cov2 = torch.empty((m, 3), dtype=torch.float64, device="cuda")
    fit = torch.empty(19, dtype=torch.float64, device="cuda") if m >= 6 else None
    native.darb_psi_calibrate(kernel, m, sig, grid_n, ws, cov2, fit)
    torch.cuda.synchronize()
    out = dict(cov2=cov2.cpu().numpy())
    if fit is not None:
        f = fit.cpu().numpy()
        out["coef"], out["psi"] = f[:18].reshape(3, 6), float(f[18])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--m", type=int, default=1000)
    ap.add_argument("--grid", type=int, default=97)
    args = ap.parse_args()
    for name, k in pipeline.KERNELS.items():
        r = calibrate_psi(k, m=args.m, grid_n=args.grid)
        print(f"{name:16s} psi={r['psi']:.4f}  a'={np.round(r['coef'][0], 3)}  b'={np.round(r['coef'][1], 3)}  "
              f"d'={np.round(r['coef'][2], 3)}", flush=True)


if __name__ == "__main__":
    main()
