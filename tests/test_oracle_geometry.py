"""Pins of the oracle's per-Gaussian geometry against mathematics the paper fixes.

R(q) (App. A, Eq. quat) against the Hamilton-product rotation; Sigma = R S S^T R^T
(Sec. 4) against its eigen-decomposition; the EWA projection (Sec. 4, Eq.
volume-render) against closed forms and a finite-difference Jacobian of the
pinhole map; culling (Sec. 6) against brute-force pixel enumeration.
"""
import math

import numpy as np
import pytest

import scenes
from oracle.gaussians import project, quaternion_to_rotation
from oracle.raster import render_bruteforce, tile_lists
from oracle.rules import Rules
from tests.helpers import dc_for_colour, logit_of, make_scene


def hamilton(a, b):
    ar, ai, aj, ak = a
    br, bi, bj, bk = b
    return np.array([ar * br - ai * bi - aj * bj - ak * bk,
                     ar * bi + ai * br + aj * bk - ak * bj,
                     ar * bj - ai * bk + aj * br + ak * bi,
                     ar * bk + ai * bj - aj * bi + ak * br])


def test_rotation_matches_hamilton_product():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((50, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    R = quaternion_to_rotation(q)
    for n in range(50):
        for e in np.eye(3):
            qc = q[n] * np.array([1, -1, -1, -1])
            rot = hamilton(hamilton(q[n], np.concatenate([[0.0], e])), qc)[1:]
            np.testing.assert_allclose(R[n] @ e, rot, atol=1e-14)
        np.testing.assert_allclose(R[n] @ R[n].T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R[n]) - 1.0) < 1e-13


def test_covariance_eigenvalues_are_squared_scales():
    rng = np.random.default_rng(1)
    n = 20
    ls = rng.normal(-1.0, 0.5, (n, 3))
    sc = make_scene(np.tile([0.0, 0.0, 5.0], (n, 1)), ls, rng.standard_normal((n, 4)),
                    np.zeros(n), np.zeros((n, 1, 3)))
    p = project(sc, scenes.pinhole_camera(64, 64))
    for k in range(n):
        ev = np.sort(np.linalg.eigvalsh(p.Sigma[k]))
        np.testing.assert_allclose(ev, np.sort(np.exp(2 * ls[k])), rtol=1e-12)


def test_isotropic_on_axis_closed_form():
    # Sigma' = diag((fx s / z0)^2, (fy s / z0)^2) for an isotropic Gaussian on the axis
    s, z0 = 0.3, 4.0
    sc = make_scene([[0.0, 0.0, z0]], np.full((1, 3), math.log(s)), [[1, 0, 0, 0]], [0.0],
                    np.zeros((1, 1, 3)))
    cam = scenes.pinhole_camera(64, 48)
    p = project(sc, cam)
    f = float(cam.fx)
    np.testing.assert_allclose(p.cov2d[0], np.diag([(f * s / z0) ** 2, (f * s / z0) ** 2]),
                               rtol=1e-13)
    assert p.u[0] == float(cam.cx) and p.v[0] == float(cam.cy)


def pinhole(cam, x):
    return np.array([float(cam.fx) * x[0] / x[2] + float(cam.cx),
                     float(cam.fy) * x[1] / x[2] + float(cam.cy)])


def test_off_axis_projection_matches_numeric_jacobian():
    # Sigma' = J W Sigma W^T J^T with J the Jacobian of the pinhole map (checked numerically)
    rng = np.random.default_rng(2)
    cam = scenes.look_at_camera([1.0, -0.5, -2.0], [0.2, 0.1, 4.0], 80, 60)
    for _ in range(10):
        mu = rng.uniform([-1, -1, 3], [1, 1, 6])
        ls = rng.normal(-1.5, 0.4, 3)
        q = rng.standard_normal(4)
        sc = make_scene([mu], [ls], [q], [0.0], np.zeros((1, 1, 3)))
        p = project(sc, cam)
        W = cam.R.astype(np.float64)
        t = W @ mu + cam.t.astype(np.float64)
        h = 1e-6
        Jn = np.stack([(pinhole(cam, t + h * e) - pinhole(cam, t - h * e)) / (2 * h)
                       for e in np.eye(3)], 1)
        Rq = quaternion_to_rotation((q / np.linalg.norm(q))[None])[0]
        Sigma = Rq @ np.diag(np.exp(2 * ls)) @ Rq.T
        ref = Jn @ W @ Sigma @ W.T @ Jn.T
        np.testing.assert_allclose(p.cov2d[0], ref, rtol=1e-7)
        np.testing.assert_allclose([p.u[0], p.v[0]], pinhole(cam, t), rtol=1e-12)


def test_axis_aligned_gaussian_on_axis_ignores_depth_scale():
    cam = scenes.pinhole_camera(32, 32)
    imgs = []
    for sz in (0.01, 0.3, 1.0):
        sc = make_scene([[0.0, 0.0, 3.0]], [[math.log(0.2), math.log(0.1), math.log(sz)]],
                        [[1, 0, 0, 0]], [logit_of(0.8)], dc_for_colour([[0.9, 0.5, 0.2]]))
        imgs.append(render_bruteforce(project(sc, cam)).color)
    np.testing.assert_array_equal(imgs[0], imgs[1])
    np.testing.assert_array_equal(imgs[0], imgs[2])


def test_quaternion_scale_invariance():
    rng = np.random.default_rng(3)
    sc, cams = scenes.workload("small", n=200)
    base = render_bruteforce(project(sc, cams[0])).color
    for lam in (-1.0, 2.5, 1e-3):
        sc2 = scenes.Scene(sc.means, sc.log_scales, (sc.quats.astype(np.float64) * lam),
                           sc.opacity_logits, sc.sh, sc.sh_degree)
        img = render_bruteforce(project(sc2, cams[0])).color
        np.testing.assert_allclose(img, base, atol=1e-12)
    del rng


def test_near_cull_and_degenerate_inputs():
    cam = scenes.pinhole_camera(32, 32)
    z_near = float(np.float32(0.2))
    mu = [[0, 0, 0.1], [0, 0, z_near], [0, 0, -3.0], [0, 0, 3.0], [0, 0, 3.0], [np.nan, 0, 3.0]]
    q = [[1, 0, 0, 0]] * 4 + [[0, 0, 0, 0], [1, 0, 0, 0]]
    sc = make_scene(mu, np.full((6, 3), math.log(0.05)), q, np.zeros(6), np.zeros((6, 1, 3)))
    p = project(sc, cam)
    assert p.valid.tolist() == [False, True, False, True, False, False]


def test_depth_key_is_monotone_float_bits():
    z = np.sort(np.random.default_rng(4).uniform(0.2, 1e4, 10000)).astype(np.float32)
    keys = z.view(np.uint32)
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)


@pytest.mark.parametrize("size", [(37, 29), (16, 16), (50, 17)])
def test_tile_membership_by_enumeration(size):
    # a Gaussian is listed in a tile iff some pixel centre of the tile is in its 3-sigma box,
    # and every pixel inside its ellipse lies in one of its tiles
    W, H = size
    sc = scenes.uniform_scene(120, 7, 0, (2.0, 5.0), log_scale_mean=math.log(0.08))
    cam = scenes.pinhole_camera(W, H)
    r = Rules()
    p = project(sc, cam, r)
    tl = tile_lists(p, r)
    T = r.tile
    for g in np.nonzero(p.valid)[0]:
        # brute-force box: pixel centres within [u - rx, u + rx] x [v - ry, v + ry]
        rx = 3 * math.sqrt(p.cov2d[g, 0, 0])
        ry = 3 * math.sqrt(p.cov2d[g, 1, 1])
        xs = [i for i in range(W) if p.u[g] - rx <= i + 0.5 <= p.u[g] + rx]
        ys = [j for j in range(H) if p.v[g] - ry <= j + 0.5 <= p.v[g] + ry]
        want = sorted({(j // T) * tl.tiles_x + i // T for i in xs for j in ys})
        got = sorted(t for t in range(tl.tiles_x * tl.tiles_y)
                     if g in tl.ids[tl.start[t]:tl.start[t + 1]])
        assert got == want, g
    # ellipse pixels are inside the listed tiles
    Q = p.conic
    for g in np.nonzero(p.valid)[0]:
        for j in range(H):
            for i in range(W):
                d = np.array([i + 0.5 - p.u[g], j + 0.5 - p.v[g]])
                if d @ Q[g] @ d <= 9.0:
                    t = (j // T) * tl.tiles_x + i // T
                    assert g in tl.ids[tl.start[t]:tl.start[t + 1]]
