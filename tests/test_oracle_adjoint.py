"""Pins of the oracle's analytic adjoint (Sec. 6 back-to-front traversal; App. A).

FP64 central finite differences of a smooth linear loss L = <w, C> on tiny scenes,
accepted only where every discrete decision (culls, 3-sigma test, alpha skip,
stop, alpha clamp, colour clamp, order) is identical at theta +- h; plus the
invariants <dL/dq, q> = 0 and, for a lone degree-0 Gaussian,
dL/dk_0 = Y_0 sum_p alpha_p w_p read off the forward image.
"""
import hashlib
import math

import numpy as np
import pytest

import scenes
from oracle.adjoint import render_backward
from oracle.gaussians import project
from oracle.raster import blend, render_bruteforce, sort_order
from oracle.rules import Rules
from tests.helpers import dc_for_colour, logit_of, make_scene, tiny_random_scene

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def render_and_fingerprint(sc, cam, rules):
    p = project(sc, cam, rules)
    ids = sort_order(p, p.drawable)
    H, W = cam.height, cam.width
    py, px = np.divmod(np.arange(H * W), W)
    r = blend(p, ids, px, py, rules, record=True)
    h = hashlib.sha1()
    for a in (p.valid, p.rgb_raw >= 0, ids):
        h.update(np.ascontiguousarray(a).tobytes())
    for (_, _, bl, _, _, _, clamped, _, _) in r.steps:
        h.update(bl.tobytes())
        h.update((clamped & bl).tobytes())
    return r.color.reshape(H, W, 3), h.hexdigest()


def with_param(sc, group, index, value):
    arrs = {g: getattr(sc, g).astype(np.float64).copy() for g in GROUPS}
    arrs[group][index] = value
    return scenes.Scene(arrs["means"], arrs["log_scales"], arrs["quats"], arrs["opacity_logits"],
                        arrs["sh"], sc.sh_degree)


@pytest.mark.parametrize("seed,degree,bg", [(0, 1, (0.0, 0.0, 0.0)), (1, 2, (0.2, 0.5, 0.1)),
                                            (2, 3, (0.0, 0.0, 0.0)), (3, 0, (1.0, 1.0, 1.0))])
def test_adjoint_matches_central_differences(seed, degree, bg):
    rules = Rules(bg=bg)
    sc, cam = tiny_random_scene(6, seed, degree)
    rng = np.random.default_rng(100 + seed)
    w = rng.standard_normal((cam.height, cam.width, 3))
    grads, _, _ = render_backward(sc, cam, w, rules, bruteforce=True)
    grads_t, _, _ = render_backward(sc, cam, w, rules)
    _, fp0 = render_and_fingerprint(sc, cam, rules)
    checked = total = 0
    for group in GROUPS:
        base = getattr(sc, group).astype(np.float64)
        np.testing.assert_allclose(grads_t[group], grads[group], rtol=1e-10, atol=1e-12)
        scale = np.abs(grads[group]).max() + 1e-12
        for index in np.ndindex(base.shape):
            total += 1
            th = base[index]
            h = 1e-6 * max(1.0, abs(th))
            cp, fpp = render_and_fingerprint(with_param(sc, group, index, th + h), cam, rules)
            cm, fpm = render_and_fingerprint(with_param(sc, group, index, th - h), cam, rules)
            if fpp != fp0 or fpm != fp0:
                continue
            fd = ((w * cp).sum() - (w * cm).sum()) / (2 * h)
            assert abs(fd - grads[group][index]) <= 2e-6 * (abs(fd) + scale), (group, index)
            checked += 1
    assert checked >= 0.8 * total


def test_quaternion_gradient_is_tangent():
    sc, cam = tiny_random_scene(6, 5, 1)
    w = np.random.default_rng(6).standard_normal((cam.height, cam.width, 3))
    g, _, _ = render_backward(sc, cam, w, bruteforce=True)
    q = sc.quats.astype(np.float64)
    np.testing.assert_allclose((g["quats"] * q).sum(0), 0.0, atol=1e-12)
    assert np.abs(g["quats"]).max() > 1e-3


def test_dc_gradient_of_lone_gaussian_from_forward_image():
    cam = scenes.pinhole_camera(24, 24)
    c = np.array([0.7, 0.4, 0.9])
    sc = make_scene([[0.05, 0.02, 2.5]], [[math.log(0.2), math.log(0.1), math.log(0.15)]],
                    [[0.8, 0.1, 0.4, -0.2]], [logit_of(0.8)], dc_for_colour(c[None, None, :]))
    w = np.random.default_rng(7).standard_normal((24, 24, 3))
    g, _, _ = render_backward(sc, cam, w, bruteforce=True)
    img = render_bruteforce(project(sc, cam)).color
    alpha = img[..., 0] / c[0]                # black background: C = alpha c
    y0 = 1.0 / (2.0 * math.sqrt(math.pi))
    want = y0 * (alpha[..., None] * w).sum((0, 1))
    np.testing.assert_allclose(g["sh"][0, :, 0], want, rtol=1e-12)


def test_culled_gaussians_get_zero_gradient():
    cam = scenes.pinhole_camera(32, 32)
    sc = make_scene([[0, 0, 0.1], [0, 0, 3.0], [0, 0, 3.0]], np.full((3, 3), math.log(0.2)),
                    [[1, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 0]], np.zeros(3),
                    dc_for_colour(np.full((3, 1, 3), 0.6)))
    w = np.ones((32, 32, 3))
    g, _, _ = render_backward(sc, cam, w, bruteforce=True)
    for k in GROUPS:
        arr = g[k]
        assert np.all(arr[..., :2] == 0), k
        assert np.any(arr[..., 2] != 0) or k == "quats"
