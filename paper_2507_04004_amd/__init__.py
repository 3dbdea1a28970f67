"""MI355X (gfx950) differentiable tile-based Gaussian-splatting rasterizer.

Hot path of Gaussian-LIC2's map optimisation and photometric tracking: projection of
anisotropic Gaussians with SH colour, alpha-max tile culling, (tile, depth) sorting,
front-to-back compositing of colour / depth / opacity, and the backward pass to every
Gaussian parameter and the SE(3) camera pose with a sparse-LiDAR depth term. Every stage is
a HIP kernel in libgs.so behind the C ABI of include/gs.h; torch supplies device memory and
streams.
"""
from . import scenes  # noqa: F401

__all__ = ["scenes", "raster", "batch", "serve", "autotune"]
