"""Photometric training loss in FP64 (oracle side; test infrastructure only).

Sec. 5.1: L = (1 - lambda) L1 + lambda L_D-SSIM with lambda = 0.2.

Readings where the paper is silent:
* images are planar [3][H][W] with values nominally in [0, 1]; L1 is the mean of
  |x - y| over the 3 H W values of one view (sign(0) = 0 in its gradient);
* SSIM is the structural similarity of Wang et al. (2004) per channel: local means,
  variances and covariance under an 11 x 11 Gaussian window of standard deviation
  1.5 (normalised to sum 1), stabilising constants C1 = 0.01^2 and C2 = 0.03^2 for
  a dynamic range of 1, the window applied at every pixel with zero values outside
  the image (no renormalisation at the borders);
* L_D-SSIM = 1 - mean SSIM over the 3 H W values;
* over several views the losses add.
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA = 0.2


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """The 2D window w[a, b] = g[a] g[b], g a sampled Gaussian normalised to sum 1."""
    r = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-r * r / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def window_filter(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """out[..., i, j] = sum_{a, b} w[a, b] img[..., i + a - r, j + b - r], zero outside."""
    r = w.shape[0] // 2
    H, W = img.shape[-2:]
    pad = np.zeros(img.shape[:-2] + (H + 2 * r, W + 2 * r))
    pad[..., r:r + H, r:r + W] = img
    out = np.zeros(img.shape, dtype=np.float64)
    for a in range(w.shape[0]):
        for b in range(w.shape[1]):
            out += w[a, b] * pad[..., a:a + H, b:b + W]
    return out


def ssim_terms(x: np.ndarray, y: np.ndarray, w: np.ndarray | None = None):
    """Local statistics and the SSIM map (Wang et al. 2004) of x against y."""
    w = gaussian_window() if w is None else w
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mx, my = window_filter(x, w), window_filter(y, w)
    exx, eyy, exy = window_filter(x * x, w), window_filter(y * y, w), window_filter(x * y, w)
    vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
    a1 = 2 * mx * my + C1
    a2 = 2 * cxy + C2
    b1 = mx * mx + my * my + C1
    b2 = vx + vy + C2
    return dict(mx=mx, my=my, a1=a1, a2=a2, b1=b1, b2=b2, ssim=(a1 * a2) / (b1 * b2))


def l1(x, y):
    """(loss, dloss/dx) of the mean absolute error of one view."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    return np.abs(d).mean(), np.sign(d) / d.size


def dssim(x, y, w: np.ndarray | None = None):
    """(loss, dloss/dx) of L_D-SSIM = 1 - mean SSIM(x, y), gradient by the chain rule.

    SSIM(q) depends on x through mu_x(q), E[x^2](q) and E[xy](q), each a window sum
    around q, so dL/dx(p) = -1/(3HW) sum_q w(p - q) [dS/dmu_x(q) + 2 x(p) dS/dE[x^2](q)
    + y(p) dS/dE[xy](q)].
    """
    w = gaussian_window() if w is None else w
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    t = ssim_terms(x, y, w)
    mx, my, a1, a2, b1, b2 = (t[k] for k in ("mx", "my", "a1", "a2", "b1", "b2"))
    den = b1 * b2
    # S = a1 a2 / (b1 b2) with a1 = 2 mx my + C1, a2 = 2 (Exy - mx my) + C2,
    # b1 = mx^2 + my^2 + C1, b2 = (Exx - mx^2) + (Eyy - my^2) + C2
    d_mx = (2 * my * a2 - 2 * my * a1) / den - a1 * a2 * (2 * mx * b2 - 2 * mx * b1) / (den * den)
    d_exx = -a1 * a2 * b1 / (den * den)
    d_exy = 2 * a1 / den
    wf = w[::-1, ::-1]     # the adjoint of a window sum is the window sum with the flipped window
    g = window_filter(d_mx, wf) + 2 * x * window_filter(d_exx, wf) + y * window_filter(d_exy, wf)
    n = x.size
    return 1.0 - t["ssim"].mean(), -g / n


def photometric(x, y, lam: float = LAMBDA, w: np.ndarray | None = None):
    """(loss, dloss/dx) of (1 - lambda) L1 + lambda L_D-SSIM for one view."""
    l, gl = l1(x, y)
    d, gd = dssim(x, y, w)
    return (1 - lam) * l + lam * d, (1 - lam) * gl + lam * gd
