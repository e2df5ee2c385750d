"""The paper's 1D signal-reconstruction experiment on the GPU (Assessing DARBFs
through 1D Simulations; the extended 1D results): mixtures of DARBF components
fitted to 1D pulses by Adam, many problems (signals x kernels x component
counts x starts) in one persistent launch of libdarb's darb_fit1d.  This
module only builds the batch and moves the buffers.

    python -m paper_2501_12369_amd.fit1d [--steps 2000]
"""
from __future__ import annotations

import argparse
import math

import numpy as np
import torch

from . import native, pipeline, scenes

SWEEP_KERNELS = ("gauss", "half_cos", "raised_cos", "sinc")


def run_batch(kernel, x: np.ndarray, targets: np.ndarray, params: np.ndarray, steps: int,
              lr=(1e-2, 1e-2, 1e-2), step0: int = 0, moments=None, keep_loss: bool = True):
    """Fit ``params`` [batch, 3, n] (mu, log sigma, a) to ``targets`` [batch, m]
    at ``x`` [m] with one kernel.  Returns (params, adam_m, adam_v, losses
    [batch, steps] or None) as numpy arrays."""
    batch, _, n = params.shape
    m = len(x)
    dev = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to(dt).cuda()
    p = dev(params)
    m1 = dev(moments[0]) if moments is not None else torch.zeros_like(p)
    m2 = dev(moments[1]) if moments is not None else torch.zeros_like(p)
    loss = torch.empty((batch, steps), dtype=torch.float32, device="cuda") if keep_loss and steps > 0 else None
    native.darb_fit1d(kernel, batch, n, m, dev(x), dev(targets), p, m1, m2, steps, step0, lr, loss=loss)
    torch.cuda.synchronize()
    out = lambda t: t.cpu().numpy() if t is not None else None
    return out(p), out(m1), out(m2), out(loss)


def sweep_batch(n_list=(5, 10), seeds=8, m: int = 1024):
    """The sweep's problems for one kernel: every pulse x component count x start;
    returns (x, targets [B, m], inits per component count, labels)."""
    x, sig = scenes.signals1d(m)
    items = []
    for name in scenes.SIGNALS_1D:
        for s in range(seeds):
            items.append((name, s))
    return x, sig, items


def run_sweep(steps: int = 2000, n_list=(5, 10), seeds: int = 8, m: int = 1024, kernels=SWEEP_KERNELS):
    """Final loss of every (kernel, n, pulse, start); each (kernel, n) group is one launch."""
    x, sig, items = sweep_batch(n_list, seeds, m)
    res = {}
    for kname in kernels:
        k = pipeline.KERNELS[kname]
        for n in n_list:
            targets = np.stack([sig[name] for name, _ in items])
            inits = np.stack([scenes.fit1d_init(1000 * n + s, n) for _, s in items])
            _, _, _, losses = run_batch(k, x, targets, inits, steps)
            res[(kname, n)] = {(name, s): float(losses[i, -1]) for i, (name, s) in enumerate(items)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    args = ap.parse_args()
    res = run_sweep(args.steps)
    for (kname, n), d in res.items():
        best = {}
        for (name, s), L in d.items():
            best[name] = min(best.get(name, math.inf), L)
        print(f"{kname:12s} n={n:2d} " + " ".join(f"{nm}={best[nm]:.2e}" for nm in scenes.SIGNALS_1D), flush=True)


if __name__ == "__main__":
    main()
