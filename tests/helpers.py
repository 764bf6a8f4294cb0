"""Small builders shared by the tests (no rasterizer arithmetic here)."""
from __future__ import annotations

import numpy as np

import scenes


def make_scene(mu, log_s, q, logit, sh, degree=None, dtype=np.float64):
    """Scene from per-Gaussian rows: mu (N,3), log_s (N,3), q (N,4), logit (N,), sh (N,K,3)."""
    mu = np.atleast_2d(np.asarray(mu, dtype=np.float64))
    n = mu.shape[0]
    sh = np.asarray(sh, dtype=np.float64).reshape(n, -1, 3)
    k = sh.shape[1]
    degree = int(round(np.sqrt(k))) - 1 if degree is None else degree
    return scenes.Scene(
        np.ascontiguousarray(mu.T.astype(dtype)),
        np.ascontiguousarray(np.asarray(log_s, dtype=np.float64).reshape(n, 3).T.astype(dtype)),
        np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(n, 4).T.astype(dtype)),
        np.ascontiguousarray(np.asarray(logit, dtype=np.float64).reshape(n).astype(dtype)),
        np.ascontiguousarray(sh.transpose(1, 2, 0).astype(dtype)), degree)


def logit_of(o):
    o = np.asarray(o, dtype=np.float64)
    return np.log(o / (1.0 - o))


def dc_for_colour(c):
    """SH DC coefficient that gives colour c at degree 0 (c = k / (2 sqrt(pi)) + 0.5)."""
    return (np.asarray(c, dtype=np.float64) - 0.5) * 2.0 * np.sqrt(np.pi)


def tiny_random_scene(n, seed, degree=1, width=32, height=32, z=(3.0, 5.0), spread=0.6,
                      log_s=(np.log(0.25), 0.3)):
    """A few big Gaussians in front of a small camera (finite-difference checks)."""
    rng = np.random.default_rng(seed)
    mu = np.stack([rng.uniform(-spread, spread, n), rng.uniform(-spread, spread, n),
                   rng.uniform(z[0], z[1], n)], 1)
    ls = rng.normal(log_s[0], log_s[1], (n, 3))
    q = rng.standard_normal((n, 4))
    logit = rng.normal(0.5, 1.0, n)
    k = (degree + 1) ** 2
    sh = np.concatenate([rng.uniform(-1, 1, (n, 1, 3)), rng.normal(0, 0.3, (n, k - 1, 3))], 1)
    cam = scenes.pinhole_camera(width, height)
    return make_scene(mu, ls, q, logit, sh, degree), cam
