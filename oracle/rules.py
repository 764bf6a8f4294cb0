"""The fixed numerical rules of the rasterizer (oracle side; test infrastructure only).

* 16x16 pixel tiles (Sec. 6 and App. C, "Sorting").
* A Gaussian reaches a pixel only inside its 3-sigma ellipse, i.e. where the
  Mahalanobis distance m = d^T Sigma'^-1 d <= 9. The paper culls against the
  99% confidence region (Sec. 6); 3 sigma holds 1 - e^-4.5 = 98.9% of a 2D
  Gaussian's mass. Applying the same test per pixel makes the image independent
  of the tile size (reading; the paper only culls per tile).
* Near cull: camera-space depth below 0.2 is rejected (the guard band of Sec. 6
  gives no numbers; 0.2 is the reading taken).
* Skip any alpha below 1/255, clamp alpha to at most 0.99, and stop a pixel
  before its accumulated opacity would exceed 0.9999, i.e. when T(1 - alpha)
  would fall below 1e-4 (App. C, "Numerical stability").

Two switches reproduce the ablations of Sec. 7.3 (both off in the method itself):
* isotropic: one scalar radius per Gaussian on all three axes, Sigma = s^2 I. The
  scalar is s = exp of the mean of the three stored log-scales (so three equal
  rows behave exactly as one parameter, each receiving a third of its gradient);
  the quaternion is not used and receives no gradient.
* grad_limit = N > 0: only the N front-most Gaussians blended at a pixel receive
  gradient from it (their gradient is the exact one); the image is unchanged.
"""
from __future__ import annotations

import dataclasses


@dataclasses.dataclass(frozen=True)
class Rules:
    tile: int = 16
    near_z: float = 0.2
    sigma_extent: float = 3.0
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    bg: tuple = (0.0, 0.0, 0.0)
    isotropic: bool = False
    grad_limit: int = 0
    # Decision margins: a pixel is "ambiguous" when one of its threshold decisions
    # lies so close to the threshold that an FP32 evaluation may legitimately take
    # the other branch. Each width is about 10x an FP32 error bound of the quantity:
    #   m      ~ 1e-6 relative (the position stored to FP32 relative to a nearby
    #          integer corner, a few roundings of terms <= 9)
    #   alpha  ~ 5e-6 relative (m error / 2 plus the exponential's error)
    #   T'     ~ (k + 4) * 6e-8 relative after k blended factors
    #   bounds ~ 1e-7 px (FP64 projection evaluated in a different order)
    margin_m: float = 1e-5        # |m - 9| < margin_m * 9
    margin_alpha: float = 5e-5    # |alpha - 1/255| < margin_alpha / 255
    margin_T_per_step: float = 6e-7   # |T' - 1e-4| < (k + 4) * this * 1e-4 after k blends
    margin_px: float = 1e-6       # AABB bound within this many pixels of an integer
