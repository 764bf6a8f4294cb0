"""Pins of the oracle's blending (Eq. front-to-back; Sec. 6; App. C and Alg. 2)."""
import math
import os

import numpy as np
import pytest

import scenes
from oracle.gaussians import project
from oracle.raster import render_bruteforce, render_tiles, tile_lists
from oracle.rules import Rules
from tests.helpers import dc_for_colour, logit_of, make_scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *vals = line.split()
        out[k] = [float(x) for x in vals]
    return out


def test_worked_example_stop_rule():
    g = read_golden("stop_rule_stack.txt")
    o = g["opacity"][0]
    cam = scenes.pinhole_camera(32, 32, cx=16.5, cy=16.5)
    n = 4
    mu = [[0.0, 0.0, z] for z in (2.0, 3.0, 4.0, 5.0)]
    sc = make_scene(mu, np.full((n, 3), math.log(0.05)), [[1, 0, 0, 0]] * n,
                    np.full(n, logit_of(o)), dc_for_colour(np.ones((n, 1, 3))))
    p = project(sc, cam)
    img = render_bruteforce(p)
    # per-Gaussian weight at that pixel, one Gaussian at a time by differencing
    np.testing.assert_allclose(img.color[16, 16], g["color"][0], rtol=1e-12)
    np.testing.assert_allclose(img.T_final[16, 16], g["T_final"][0], rtol=1e-12)
    assert img.last_id[16, 16] == int(g["last_contributor"][0])
    w = []
    for k in range(n):
        sub = make_scene(mu[:k + 1], np.full((k + 1, 3), math.log(0.05)), [[1, 0, 0, 0]] * (k + 1),
                         np.full(k + 1, logit_of(o)), dc_for_colour(np.ones((k + 1, 1, 3))))
        w.append(render_bruteforce(project(sub, cam)).color[16, 16, 0])
    weights = np.diff([0.0] + w)
    np.testing.assert_allclose(weights, g["weight"], atol=1e-15)


def test_weights_and_final_T_sum_to_one():
    # all colours 1, black background: image = sum_i T_i alpha_i = 1 - T_final
    sc, cams = scenes.workload("small", n=400)
    sc = scenes.Scene(sc.means, sc.log_scales, sc.quats, sc.opacity_logits,
                      dc_for_colour(np.ones((1, 3, sc.n))), 0)
    img = render_bruteforce(project(sc, cams[0]))
    np.testing.assert_allclose(img.color, (1.0 - img.T_final)[..., None] * np.ones(3), atol=1e-13)


def test_single_gaussian_closed_form():
    cam = scenes.pinhole_camera(24, 20)
    c = np.array([0.8, 0.3, 0.6])
    bg = (0.1, 0.2, 0.3)
    r = Rules(bg=bg)
    sc = make_scene([[0.1, -0.05, 2.0]], [[math.log(0.15), math.log(0.08), math.log(0.1)]],
                    [[0.9, 0.2, -0.3, 0.1]], [logit_of(0.7)], dc_for_colour(c[None, None, :]))
    p = project(sc, cam, r)
    img = render_bruteforce(p, r)
    Q = p.conic[0]
    for j in range(cam.height):
        for i in range(cam.width):
            d = np.array([i + 0.5 - p.u[0], j + 0.5 - p.v[0]])
            m = d @ Q @ d
            a = min(0.99, 0.7 * math.exp(-0.5 * m))
            if m <= 9 and a >= 1 / 255:
                want = a * c + (1 - a) * np.array(bg)
            else:
                want = np.array(bg)
            np.testing.assert_allclose(img.color[j, i], want, atol=1e-12)


def test_alpha_clamp_and_skip():
    cam = scenes.pinhole_camera(32, 32, cx=16.5, cy=16.5)
    # opacity ~1 at the centre: alpha clamps to 0.99
    sc = make_scene([[0.0, 0.0, 3.0]], np.full((1, 3), math.log(0.2)), [[1, 0, 0, 0]],
                    [logit_of(0.999999)], dc_for_colour(np.ones((1, 1, 3))))
    img = render_bruteforce(project(sc, cam))
    np.testing.assert_allclose(img.color[16, 16, 0], 0.99, rtol=1e-14)
    # opacity below 1/255 everywhere: nothing is blended
    sc = make_scene([[0.0, 0.0, 3.0]], np.full((1, 3), math.log(0.2)), [[1, 0, 0, 0]],
                    [logit_of(0.9 / 255)], dc_for_colour(np.ones((1, 1, 3))))
    img = render_bruteforce(project(sc, cam))
    assert np.all(img.color == 0) and np.all(img.last_id == -1)


def test_front_gaussian_occludes():
    cam = scenes.pinhole_camera(32, 32, cx=16.5, cy=16.5)
    sc = make_scene([[0.0, 0.0, 4.0], [0.0, 0.0, 2.0]], np.full((2, 3), math.log(0.3)),
                    [[1, 0, 0, 0]] * 2, [logit_of(0.9)] * 2,
                    dc_for_colour(np.array([[[1.0, 0, 0]], [[0, 1.0, 0]]])))
    img = render_bruteforce(project(sc, cam))
    px = img.color[16, 16]
    assert img.last_id[16, 16] == 0           # the far one (id 0) is blended last
    np.testing.assert_allclose(px, [0.1 * 0.9, 0.9, 0.0], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("size,n,seed", [((128, 128), 1000, 0), ((37, 29), 300, 3),
                                         ((50, 17), 200, 4)])
def test_bruteforce_equals_binned(size, n, seed):
    sc = scenes.uniform_scene(n, seed, 1, (2.0, 6.0))
    cam = scenes.pinhole_camera(*size)
    p = project(sc, cam)
    a = render_bruteforce(p)
    b = render_tiles(p)
    np.testing.assert_array_equal(a.color, b.color)
    np.testing.assert_array_equal(a.T_final, b.T_final)
    np.testing.assert_array_equal(a.last_id, b.last_id)


@pytest.mark.parametrize("tile", [8, 32])
def test_image_independent_of_tile_size(tile):
    sc = scenes.uniform_scene(500, 9, 1, (2.0, 6.0))
    cam = scenes.pinhole_camera(70, 45)
    p16 = project(sc, cam)
    base = render_tiles(p16)
    r = Rules(tile=tile)
    other = render_tiles(project(sc, cam, r), r)
    np.testing.assert_array_equal(base.color, other.color)
    tl = tile_lists(project(sc, cam, r), r)
    assert tl.tiles_x == math.ceil(70 / tile)


def test_depth_tie_broken_by_index():
    cam = scenes.pinhole_camera(32, 32, cx=16.5, cy=16.5)
    sc = make_scene([[0.0, 0.0, 3.0], [0.0, 0.0, 3.0]], np.full((2, 3), math.log(0.3)),
                    [[1, 0, 0, 0]] * 2, [logit_of(0.6)] * 2,
                    dc_for_colour(np.array([[[1.0, 0, 0]], [[0, 1.0, 0]]])))
    img = render_bruteforce(project(sc, cam))
    np.testing.assert_allclose(img.color[16, 16], [0.6, 0.4 * 0.6, 0], rtol=1e-12, atol=1e-15)
    tl = tile_lists(project(sc, cam))
    assert list(tl.ids[tl.start[0]:tl.start[1]]) == [0, 1]
