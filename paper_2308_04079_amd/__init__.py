"""MI355X-native (gfx950) differentiable tile rasterizer for 3D Gaussian splats.

The hot path of Kerbl et al., "3D Gaussian Splatting for Real-Time Radiance Field
Rendering" (SIGGRAPH 2023): projection, binning, radix sort, front-to-back blending
and the matching backward pass, as hand-written HIP kernels behind the C ABI of
include/gs.h (libgs_mi355x.so). This package is the thin Python layer above it.
"""
from .raster import GaussianParams, Rasterizer, RasterizeFunction, RenderState, rasterize  # noqa: F401
