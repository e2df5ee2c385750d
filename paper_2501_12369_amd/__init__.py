"""MI355X (gfx950) differentiable DARBF splatting rasterizer (DARB-Splatting,
arXiv 2501.12369): HIP kernels behind the C ABI of ``include/darb.h``.

Submodules are imported lazily so that ``scenes`` (seeded inputs) can be used
without loading the library; the rasterizer modules fail loudly if
``libdarb.so`` is missing.
"""

__all__ = ["native", "pipeline", "autograd", "scenes", "build"]
