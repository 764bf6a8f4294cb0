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
* isotropic: one radius on all three axes per Gaussian, Sigma = s^2 I. The
  scalar is s = exp of the mean of the three stored log-scales (so three equal
  rows behave exactly as one parameter, each receiving a third of its gradient);
  the quaternion is not used and receives no gradient.
* grad_limit = N > 0: only the N front-most Gaussians blended at a pixel receive
  gradient from it (their gradient is the exact one); the image is unchanged.

Decision margins. The thresholds (m <= 9, alpha >= 1/255, T' >= 1e-4, the alpha
clamp, the pixel-box bounds) are sharp, so an FP32 evaluation of the same
quantities may legitimately take the other branch where the exact value lies
close to a threshold. The oracle therefore carries, for every decision, a
first-order bound on the rounding error of an FP32 evaluation of that quantity
from FP32-stored inputs (the inverse covariance in its whitened (Cholesky) form
L^-1, the whitened offset of the centre of the pixel box's corner pixel from the 2D
mean, the opacity; m as the squared norm of L^-1 D plus that offset, D the exact
pixel offset from the corner; the exponential good to a few units in the last
place; the running product T),
and flags the decision when the exact value lies within that bound of the
threshold, times a scale per kind of decision. Each scale is set so
that the margin is at least ten times the worst FP32 error measured against this
oracle, as a fraction of the same bound: on the test workloads an IEEE binary32
evaluation of m from the FP32-stored inputs reaches 0.83 of its bound, of alpha
0.59, of the running product T 0.27.
"""
from __future__ import annotations

import dataclasses

EPS32 = 2.0 ** -24   # unit roundoff of IEEE binary32


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
    margin_m: float = 10.0        # margin of m <= ext^2: this x its FP32 error bound
    margin_alpha: float = 6.0     # margin of alpha >= alpha_min and of the alpha clamp
    margin_T: float = 3.0         # margin of T' >= T_min
    margin_px: float = 1e-6       # AABB bound within this many pixels of an integer
