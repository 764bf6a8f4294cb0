"""FP64 CPU oracle for the tile rasterizer of 3D Gaussian Splatting (Kerbl et al. 2023).

TEST INFRASTRUCTURE, NOT PRODUCT. Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package. The HIP library never calls it, links it or falls back to it, and this
package imports nothing from the HIP side: the two share only the seeded input
arrays produced by the ``scenes`` module.

Plain, slow, obviously-correct NumPy in float64. Every function cites the paper
passage it follows. Where the paper is silent the reading taken is written next
to the code (camera model, SH basis, per-pixel 3-sigma extent, stop rule, ...).

Modules
-------
rules      the fixed numerical rules (tile size, near cull, 3-sigma, alpha rules)
gaussians  activation, R(q), Sigma, view transform, EWA projection, SH colour
raster     depth keys, tile lists, front-to-back blending (brute force and binned)
adjoint    the analytic reverse-mode derivative of everything above
"""
from .rules import Rules  # noqa: F401
from .gaussians import project, sh_basis, quaternion_to_rotation  # noqa: F401
from .raster import (tile_lists, render_bruteforce, render_tiles,  # noqa: F401
                     sort_order)
from .adjoint import render_backward  # noqa: F401
