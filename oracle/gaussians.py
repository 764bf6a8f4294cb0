"""Per-Gaussian forward quantities in FP64 (oracle side; test infrastructure only).

Follows Sec. 4 (Sigma = R S S^T R^T; Sigma' = J W Sigma W^T J^T keeping the upper
2x2), Sec. 5.1 (sigmoid opacity, exponential scale activation), App. A Eq. (quat)
for R(q), and Sec. 6 for culling. Readings taken where the paper is silent:

* camera: pinhole, OpenCV axes (x right, y down, z forward), world-to-camera
  [W | t], pixel (i, j) has its centre at (i + 0.5, j + 0.5);
* J is the 2x3 Jacobian of (fx x/z + cx, fy y/z + cy) at the camera-space mean;
  no screen-space low-pass dilation is added to Sigma';
* the depth sorted on is z32, the float32 rounding of the float64 value
  ((W20 x + W21 y) + W22 z) + t2 evaluated in exactly that order without fused
  multiply-add; the near cull compares z32 with float32(0.2);
* colour is max(sum_lm k_lm Y_lm(d) + 0.5, 0) per channel with real orthonormal
  SH without the Condon-Shortley phase and d the unit vector from the camera
  centre to the mean, in world space.
"""
from __future__ import annotations

import dataclasses
from math import comb, factorial, pi, sqrt

import numpy as np

from .rules import Rules


def quaternion_to_rotation(q: np.ndarray) -> np.ndarray:
    """R(q) of a unit quaternion q = (r, i, j, k): App. A, Eq. (quat). q: (N, 4) -> (N, 3, 3)."""
    r, i, j, k = (q[:, c] for c in range(4))
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1.0 - 2.0 * (j * j + k * k)
    R[:, 0, 1] = 2.0 * (i * j - r * k)
    R[:, 0, 2] = 2.0 * (i * k + r * j)
    R[:, 1, 0] = 2.0 * (i * j + r * k)
    R[:, 1, 1] = 1.0 - 2.0 * (i * i + k * k)
    R[:, 1, 2] = 2.0 * (j * k - r * i)
    R[:, 2, 0] = 2.0 * (i * k - r * j)
    R[:, 2, 1] = 2.0 * (j * k + r * i)
    R[:, 2, 2] = 1.0 - 2.0 * (i * i + j * j)
    return R


# ---------------------------------------------------------------------------
# Real spherical harmonics as polynomials in the unit direction (x, y, z).
# Built from the general closed form of the real regular solid harmonics
# (Legendre part Pi_l^m(z, r) times the planar parts A_m = Re (x + i y)^m and
# B_m = Im (x + i y)^m), normalised to be orthonormal on the sphere. The paper
# names SH colour (Sec. 3, Sec. 5) but fixes no basis: this is the reading.
# Coefficient index k = l^2 + l + m.
# ---------------------------------------------------------------------------

def _poly_mul(p, q):
    out = {}
    for (a1, b1, c1), v1 in p.items():
        for (a2, b2, c2), v2 in q.items():
            key = (a1 + a2, b1 + b2, c1 + c2)
            out[key] = out.get(key, 0.0) + v1 * v2
    return out


def _r2_pow(k):
    p = {(0, 0, 0): 1.0}
    r2 = {(2, 0, 0): 1.0, (0, 2, 0): 1.0, (0, 0, 2): 1.0}
    for _ in range(k):
        p = _poly_mul(p, r2)
    return p


def _planar(m, use_sin):
    """A_m (cos) or B_m (sin): sum_p C(m,p) x^p y^(m-p) {cos, sin}((m - p) pi / 2)."""
    cos4 = (1.0, 0.0, -1.0, 0.0)
    sin4 = (0.0, 1.0, 0.0, -1.0)
    out = {}
    for p in range(m + 1):
        f = (sin4 if use_sin else cos4)[(m - p) % 4]
        if f != 0.0:
            out[(p, m - p, 0)] = out.get((p, m - p, 0), 0.0) + comb(m, p) * f
    return out


def sh_polynomials(degree: int):
    polys = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            leg = {}
            for k in range((l - am) // 2 + 1):
                c = ((-1) ** k) * 2.0 ** (-l) * comb(l, k) * comb(2 * l - 2 * k, l) \
                    * factorial(l - 2 * k) / factorial(l - 2 * k - am)
                for (a, b, cc), v in _r2_pow(k).items():
                    key = (a, b, cc + l - 2 * k - am)
                    leg[key] = leg.get(key, 0.0) + c * v
            norm = sqrt((2 * l + 1) / (4.0 * pi) * factorial(l - am) / factorial(l + am))
            if m == 0:
                planar, f = {(0, 0, 0): 1.0}, 1.0
            else:
                planar, f = _planar(am, use_sin=(m < 0)), sqrt(2.0)
            poly = {key: norm * f * v for key, v in _poly_mul(leg, planar).items()}
            polys.append(poly)
    return polys


def sh_basis(degree: int, dirs: np.ndarray) -> np.ndarray:
    """Y_k(d) for unit directions dirs (N, 3) -> (N, K)."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    polys = sh_polynomials(degree)
    out = np.zeros((dirs.shape[0], len(polys)))
    for k, poly in enumerate(polys):
        for (a, b, c), v in poly.items():
            out[:, k] += v * x ** a * y ** b * z ** c
    return out


def sh_basis_grad(degree: int, dirs: np.ndarray) -> np.ndarray:
    """dY_k/d(x, y, z) of the polynomials at dirs (N, 3) -> (N, K, 3)."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    polys = sh_polynomials(degree)
    out = np.zeros((dirs.shape[0], len(polys), 3))
    for k, poly in enumerate(polys):
        for (a, b, c), v in poly.items():
            if a:
                out[:, k, 0] += v * a * x ** (a - 1) * y ** b * z ** c
            if b:
                out[:, k, 1] += v * b * x ** a * y ** (b - 1) * z ** c
            if c:
                out[:, k, 2] += v * c * x ** a * y ** b * z ** (c - 1)
    return out


@dataclasses.dataclass
class Projection:
    """Everything the oracle knows about each Gaussian in one view (FP64 unless noted)."""
    n: int
    valid: np.ndarray       # (N,) bool: survives every cull
    drawable: np.ndarray    # (N,) bool: survives every cull except the empty-AABB one
    z32: np.ndarray         # (N,) float32 sort depth
    zkey: np.ndarray        # (N,) uint32 bit pattern of z32
    u: np.ndarray
    v: np.ndarray
    cov2d: np.ndarray       # (N, 2, 2) Sigma'
    conic: np.ndarray       # (N, 2, 2) Sigma'^-1
    i_lo: np.ndarray
    i_hi: np.ndarray
    j_lo: np.ndarray
    j_hi: np.ndarray
    tx0: np.ndarray
    tx1: np.ndarray
    ty0: np.ndarray
    ty1: np.ndarray
    opacity: np.ndarray
    rgb: np.ndarray         # (N, 3) clamped colour
    rgb_raw: np.ndarray     # (N, 3) before the clamp at 0
    aabb_margin: np.ndarray  # (N,) bool: a pixel bound lies within margin_px of an integer
    # intermediates kept for the adjoint
    s: np.ndarray
    qhat: np.ndarray
    qnorm: np.ndarray
    R: np.ndarray
    M: np.ndarray
    Sigma: np.ndarray
    t: np.ndarray           # (N, 3) camera-space mean (t_z = z64)
    J: np.ndarray           # (N, 2, 3)
    W: np.ndarray           # (3, 3) view rotation
    dirs: np.ndarray        # (N, 3) unit SH direction
    dist: np.ndarray        # (N,) |mu - camera centre|
    shY: np.ndarray         # (N, K)
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    sh_degree: int
    isotropic: bool = False  # Sigma = s^2 I with s = exp(mean log-scale)


def project(scene, cam, rules: Rules = Rules()) -> Projection:
    """Activation, view transform, culling, EWA projection and SH colour of every Gaussian."""
    n = scene.n
    mu = scene.means.astype(np.float64).T              # (N, 3)
    log_s = scene.log_scales.astype(np.float64).T
    q = scene.quats.astype(np.float64).T
    logit = scene.opacity_logits.astype(np.float64)
    sh = scene.sh.astype(np.float64)                    # (K, 3, N)
    W = cam.R.astype(np.float64)
    tw = cam.t.astype(np.float64)
    fx, fy, cx, cy = (float(np.float64(a)) for a in (cam.fx, cam.fy, cam.cx, cam.cy))
    Wd, Hd = cam.width, cam.height

    with np.errstate(all="ignore"):
        finite = np.isfinite(mu).all(1) & np.isfinite(log_s).all(1) & np.isfinite(logit) \
            & np.isfinite(sh).all(axis=(0, 1))
        if rules.isotropic:
            # one radius on all axes (Sec. 7.3 ablation): no rotation, q unused
            s = np.repeat(np.exp(log_s.mean(1))[:, None], 3, 1)
            q = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
        else:
            finite &= np.isfinite(q).all(1)
            # activations (Sec. 5.1): s = exp(log s); q normalised (Sec. 4)
            s = np.exp(log_s)
        o = 1.0 / (1.0 + np.exp(-logit))
        qnorm = np.sqrt((q * q).sum(1))
        ok_q = finite & (qnorm > 0)
        qhat = np.where(ok_q[:, None], q / np.where(qnorm > 0, qnorm, 1.0)[:, None], 0.0)
        R = quaternion_to_rotation(qhat)
        M = R * s[:, None, :]                           # M = R S (column j scaled by s_j)
        Sigma = M @ M.transpose(0, 2, 1)                # Sigma = M M^T (Sec. 4)

        # view transform, componentwise in a fixed order without fusion
        t = np.empty((n, 3))
        for r in range(3):
            t[:, r] = ((W[r, 0] * mu[:, 0] + W[r, 1] * mu[:, 1]) + W[r, 2] * mu[:, 2]) + tw[r]
        z32 = t[:, 2].astype(np.float32)
        near_ok = z32 >= np.float32(rules.near_z)

        tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
        u = fx * tx / tz + cx
        v = fy * ty / tz + cy
        J = np.zeros((n, 2, 3))
        J[:, 0, 0] = fx / tz
        J[:, 0, 2] = -fx * tx / (tz * tz)
        J[:, 1, 1] = fy / tz
        J[:, 1, 2] = -fy * ty / (tz * tz)
        U = J @ W                                        # U = J W (App. A)
        cov2d = U @ Sigma @ U.transpose(0, 2, 1)         # Eq. (volume-render), upper 2x2
        a, b, c = cov2d[:, 0, 0], cov2d[:, 0, 1], cov2d[:, 1, 1]
        det = a * c - b * b
        det_ok = np.isfinite(det) & (det > 0) & np.isfinite(u) & np.isfinite(v)
        conic = np.empty((n, 2, 2))
        conic[:, 0, 0] = c / det
        conic[:, 0, 1] = -b / det
        conic[:, 1, 0] = -b / det
        conic[:, 1, 1] = a / det

        # pixel AABB of the 3-sigma ellipse: pixel i is inside iff its centre i + 0.5
        # lies in [u - rx, u + rx]
        k = rules.sigma_extent
        rx = k * np.sqrt(a)
        ry = k * np.sqrt(c)
        bx0, bx1 = u - rx - 0.5, u + rx - 0.5
        by0, by1 = v - ry - 0.5, v + ry - 0.5
        ok_b = det_ok & np.isfinite(bx0) & np.isfinite(bx1) & np.isfinite(by0) & np.isfinite(by1)
        big = 1e9
        i_lo = np.maximum(0, np.ceil(np.clip(bx0, -big, big))).astype(np.int64)
        i_hi = np.minimum(Wd - 1, np.floor(np.clip(bx1, -big, big))).astype(np.int64)
        j_lo = np.maximum(0, np.ceil(np.clip(by0, -big, big))).astype(np.int64)
        j_hi = np.minimum(Hd - 1, np.floor(np.clip(by1, -big, big))).astype(np.int64)
        nonempty = (i_lo <= i_hi) & (j_lo <= j_hi)

        def near_int(x):
            return np.abs(x - np.round(x)) < rules.margin_px
        aabb_margin = near_int(bx0) | near_int(bx1) | near_int(by0) | near_int(by1)

        valid = ok_q & near_ok & ok_b & nonempty
        T = rules.tile
        tx0, tx1 = i_lo // T, i_hi // T
        ty0, ty1 = j_lo // T, j_hi // T

        # SH colour (Sec. 3, Sec. 5); direction from the camera centre -W^T t to the mean
        cam_centre = -(W.T @ tw)
        dvec = mu - cam_centre
        dist = np.sqrt((dvec * dvec).sum(1))
        dirs = dvec / np.where(dist > 0, dist, 1.0)[:, None]
        Y = sh_basis(scene.sh_degree, dirs)             # (N, K)
        rgb_raw = np.einsum("nk,kcn->nc", Y, sh) + 0.5
        rgb = np.maximum(rgb_raw, 0.0)
        drawable = ok_q & near_ok & ok_b & np.isfinite(rgb).all(1) & (dist > 0)
        valid &= drawable

    zkey = z32.view(np.uint32)
    return Projection(n, valid, drawable, z32, zkey, u, v, cov2d, conic, i_lo, i_hi, j_lo, j_hi,
                      tx0, tx1, ty0, ty1, o, rgb, rgb_raw, aabb_margin & valid,
                      s, qhat, qnorm, R, M, Sigma, t, J, W, dirs, dist, Y,
                      Wd, Hd, fx, fy, cx, cy, scene.sh_degree, bool(rules.isotropic))
