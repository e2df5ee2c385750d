"""The calibration probes compute what the benchmark's ceilings assume: the copy
copies, the fill writes zeros, and the FMA chains give the values of the same
recurrence evaluated on the CPU (the flop count the benchmark divides by)."""
import numpy as np
import pytest
import torch

from paper_2501_12369_amd import native

pytestmark = pytest.mark.gpu


def test_probe_copy_and_fill():
    print("probe copy/fill", flush=True)
    n = (1 << 20) + 12
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.full_like(src, -1.0)
    native.darb_probe_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    native.darb_probe_fill(dst)
    torch.cuda.synchronize()
    assert not dst.any()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_probe_fma_values(dtype):
    print(f"probe fma {dtype}", flush=True)
    lanes, iters = 1000, 37
    out = torch.empty(lanes, dtype=dtype, device="cuda")
    chains = native.darb_probe_fma(out, iters)
    torch.cuda.synchronize()
    assert chains == 8
    # lane i, chain k starts at (i + k) 1e-9 and runs a <- a x + y
    i = np.arange(lanes, dtype=np.float64)[:, None]
    a = (i + np.arange(chains)[None, :]) * 1e-9
    for _ in range(iters):
        a = a * 0.999 + 1e-3
    ref = a.sum(axis=1)
    got = out.cpu().numpy().astype(np.float64)
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    assert np.allclose(got, ref, rtol=tol, atol=0), np.max(np.abs(got - ref) / ref)
