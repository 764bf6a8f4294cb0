"""Seeded synthetic scenes and cameras for the tile rasterizer.

This module holds none of the rasterizer's arithmetic: only random draws and the
construction of pinhole cameras. Both the FP64 CPU oracle and the HIP path read
the FP32 arrays it produces, so the two sides see bit-identical inputs.

Recipe (every draw is FP64 from ``numpy.random.default_rng(seed)``, in the order
written, then cast once to FP32):

* uniform scenes (the 1k / 100k workloads): x, y ~ U[-1, 1], z ~ U[z_lo, z_hi];
  log-scales ~ N(ln s0, sd) per axis; quaternions ~ N(0, 1)^4 normalised;
  opacity logits ~ N(0, sd_logit); SH DC ~ U[-1, 1]; higher SH bands ~ N(0, 0.1).
* clustered scenes (the 1M / 3M workloads): 256 cluster centres
  ~ U([-10, 10]^2 x [2, 22]); per cluster a random rotation (QR of a N(0,1) 3x3 matrix) and axis
  standard deviations 1.0 * U[0.1, 1]^3 (axis ratio <= 10:1); 90% of the points get
  equal-weight cluster labels and mu = c + R diag(a) N(0, I); 10% background points
  at (0, 0, 12) + 50 * normalize(N(0, I)) (a sphere shell of radius 50);
  log-scales ~ N(ln 0.01, 0.7); logits ~ N(0, 1.5); SH as above.
* cameras: OpenCV pinhole axes (x right, y down, z forward), world-to-camera
  [R | t], 60 degree vertical field of view, f = (H / 2) / tan(30 deg),
  principal point at the image centre.

Parameter layout is structure-of-arrays, the layout the GPU reads:
means [3][N], log_scales [3][N], quats [4][N] (r, i, j, k), opacity_logits [N],
sh [K][3][N] with K = (degree + 1)^2 coefficients per colour channel.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Camera", "Scene", "pinhole_camera", "look_at_camera", "orbit_cameras",
    "uniform_scene", "clustered_scene", "jitter_means", "workload",
]


@dataclasses.dataclass
class Camera:
    """World-to-camera pinhole view. All floating fields are FP32."""
    R: np.ndarray          # (3, 3) float32, row-major rotation (world -> camera)
    t: np.ndarray          # (3,) float32 translation
    fx: np.float32
    fy: np.float32
    cx: np.float32
    cy: np.float32
    width: int
    height: int


@dataclasses.dataclass
class Scene:
    """Raw (pre-activation) Gaussian parameters, SoA FP32."""
    means: np.ndarray           # (3, N)
    log_scales: np.ndarray      # (3, N)
    quats: np.ndarray           # (4, N)  (r, i, j, k)
    opacity_logits: np.ndarray  # (N,)
    sh: np.ndarray              # (K, 3, N)
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[:, idx].copy(), self.log_scales[:, idx].copy(),
                     self.quats[:, idx].copy(), self.opacity_logits[idx].copy(),
                     self.sh[:, :, idx].copy(), self.sh_degree)


def _f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


def pinhole_camera(width: int, height: int, fov_y_deg: float = 60.0,
                   R=None, t=None, cx=None, cy=None) -> Camera:
    f = (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    R = np.eye(3) if R is None else np.asarray(R, dtype=np.float64)
    t = np.zeros(3) if t is None else np.asarray(t, dtype=np.float64)
    return Camera(_f32(R), _f32(t), np.float32(f), np.float32(f),
                  np.float32(width / 2.0 if cx is None else cx),
                  np.float32(height / 2.0 if cy is None else cy), int(width), int(height))


def look_at_camera(eye, target, width: int, height: int, fov_y_deg: float = 60.0,
                   down=(0.0, 1.0, 0.0)) -> Camera:
    """Camera at ``eye`` looking at ``target``; image y follows the world ``down`` vector."""
    eye = np.asarray(eye, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(np.asarray(down, dtype=np.float64), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return pinhole_camera(width, height, fov_y_deg, R=R, t=-R @ eye)


ORBIT_RESOLUTIONS = ((640, 360), (960, 540), (1280, 720), (1920, 1080))


def orbit_cameras(n: int, seed: int, centre=(0.0, 0.0, 12.0), radius: float = 8.0,
                  resolutions=ORBIT_RESOLUTIONS, max_elev_deg: float = 20.0):
    """Seeded orbit: eye = centre + r (cos th cos ph, sin th, cos th sin ph), looking at centre.

    Draw order: phi ~ U[0, 2 pi)^n, theta ~ U[-20, 20] deg ^n, resolution index ~ U{0..len-1}^n.
    """
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    th = np.radians(rng.uniform(-max_elev_deg, max_elev_deg, n))
    ridx = rng.integers(0, len(resolutions), n)
    c = np.asarray(centre, dtype=np.float64)
    cams = []
    for k in range(n):
        eye = c + radius * np.array([math.cos(th[k]) * math.cos(phi[k]), math.sin(th[k]),
                                     math.cos(th[k]) * math.sin(phi[k])])
        w, h = resolutions[int(ridx[k])]
        cams.append(look_at_camera(eye, c, w, h))
    return cams


def _quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _sh(rng, n, degree):
    k = (degree + 1) ** 2
    sh = np.zeros((k, 3, n))
    sh[0] = rng.uniform(-1.0, 1.0, (n, 3)).T
    if k > 1:
        sh[1:] = rng.normal(0.0, 0.1, (n, k - 1, 3)).transpose(1, 2, 0)
    return sh


def uniform_scene(n: int, seed: int, sh_degree: int = 0, z_range=(2.0, 6.0),
                  xy_range=(-1.0, 1.0), log_scale_mean=math.log(0.05),
                  log_scale_std=0.5, logit_std=1.0) -> Scene:
    rng = np.random.default_rng(seed)
    x = rng.uniform(xy_range[0], xy_range[1], n)
    y = rng.uniform(xy_range[0], xy_range[1], n)
    z = rng.uniform(z_range[0], z_range[1], n)
    ls = rng.normal(log_scale_mean, log_scale_std, (n, 3))
    q = _quats(rng, n)
    logit = rng.normal(0.0, logit_std, n)
    sh = _sh(rng, n, sh_degree)
    return Scene(_f32(np.stack([x, y, z])), _f32(ls.T), _f32(q.T), _f32(logit), _f32(sh),
                 sh_degree)


def clustered_scene(n: int, seed: int, sh_degree: int = 3, n_clusters: int = 256,
                    bg_frac: float = 0.1) -> Scene:
    rng = np.random.default_rng(seed)
    centres = np.stack([rng.uniform(-10, 10, n_clusters), rng.uniform(-10, 10, n_clusters),
                        rng.uniform(2, 22, n_clusters)], axis=1)
    # random cluster frames: QR of a Gaussian matrix, sign-fixed to a proper rotation
    a = rng.standard_normal((n_clusters, 3, 3))
    qm, rm = np.linalg.qr(a)
    qm = qm * np.sign(np.diagonal(rm, axis1=1, axis2=2))[:, None, :]
    qm[np.linalg.det(qm) < 0, :, 0] *= -1.0
    crot = qm
    axes = 1.0 * rng.uniform(0.1, 1.0, (n_clusters, 3))
    n_bg = int(round(n * bg_frac))
    n_cl = n - n_bg
    labels = rng.integers(0, n_clusters, n_cl)
    local = rng.standard_normal((n_cl, 3)) * axes[labels]
    mu_cl = centres[labels] + np.einsum("nij,nj->ni", crot[labels], local)
    d = rng.standard_normal((n_bg, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    mu_bg = np.array([0.0, 0.0, 12.0]) + 50.0 * d
    mu = np.concatenate([mu_cl, mu_bg], axis=0)
    ls = rng.normal(math.log(0.01), 0.7, (n, 3))
    q = _quats(rng, n)
    logit = rng.normal(0.0, 1.5, n)
    sh = _sh(rng, n, sh_degree)
    return Scene(_f32(mu.T), _f32(ls.T), _f32(q.T), _f32(logit), _f32(sh), sh_degree)


def jitter_means(scene: Scene, seed: int, sd: float = 0.01) -> Scene:
    """Copy of ``scene`` with means + N(0, sd) (the L1-target scene)."""
    rng = np.random.default_rng(seed + 1000)
    mu = scene.means.astype(np.float64) + rng.normal(0.0, sd, (scene.n, 3)).T
    return Scene(_f32(mu), scene.log_scales.copy(), scene.quats.copy(),
                 scene.opacity_logits.copy(), scene.sh.copy(), scene.sh_degree)


def workload(name: str, n: int | None = None):
    """The five named workloads: returns (scene, [cameras]).

    small:     1k Gaussians, SH0, 128x128, uniform z in [2, 6]
    single720: 100k Gaussians, SH3, 1280x720, uniform z in [2, 20]
    full1080:  3M Gaussians, SH3, 1920x1080, clustered scene
    multiview: 1M Gaussians clustered, 16 orbit cameras of mixed resolution
    train4:    3M Gaussians clustered, 4 orbit cameras at 1920x1080 (one step's batch)
    """
    if name == "small":
        return uniform_scene(n or 1000, 0, 0, (2.0, 6.0)), [pinhole_camera(128, 128)]
    if name == "single720":
        return uniform_scene(n or 100_000, 1, 3, (2.0, 20.0)), [pinhole_camera(1280, 720)]
    if name == "full1080":
        return clustered_scene(n or 3_000_000, 2, 3), [pinhole_camera(1920, 1080)]
    if name == "multiview":
        return clustered_scene(n or 1_000_000, 3, 3), orbit_cameras(16, 3)
    if name == "train4":
        return clustered_scene(n or 3_000_000, 4, 3), orbit_cameras(4, 4, resolutions=((1920, 1080),))
    raise KeyError(name)
