"""The blending rules of App. C ("Numerical stability") on the GPU, on stacks built so
that each rule decides the result: the worked stop-rule example of
tests/golden/stop_rule_stack.txt, and a stack whose front Gaussian is clamped at
alpha = 0.99 over the whole image (no gradient may reach its opacity or its
geometry through alpha, while its colour and the transmittance behind it still
carry gradient)."""
import math
import os

import numpy as np
import pytest

import scenes
from oracle.adjoint import render_backward
from oracle.gaussians import project
from oracle.raster import render_tiles, tile_lists
from tests.gpu_common import (GROUPS, check_grads, check_view_image, gpu_images, gpu_render,
                              to_np)
from tests.helpers import dc_for_colour, logit_of, make_scene

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, *vals = line.split()
            out[k] = [float(x) for x in vals]
    return out


def screen_grads(sc, cams, seed, state_and_rast=None):
    import torch
    rast, params, state = gpu_render(sc, cams)
    cam = cams[0]
    w = np.random.default_rng(seed).standard_normal((cam.height, cam.width, 3))
    dimg = torch.from_numpy(np.ascontiguousarray(w.transpose(2, 0, 1)).astype(np.float32))
    grads, grad2d = rast.backward(params, state, dimg.reshape(-1).cuda())
    torch.cuda.synchronize()
    gref, acc, p = render_backward(sc, cam, w)
    g2 = to_np(grad2d).reshape(-1, 9)[:sc.n].astype(np.float64)
    return state, grads, g2, gref, acc, p


def test_worked_stop_rule_stack():
    g = read_golden("stop_rule_stack.txt")
    o = g["opacity"][0]
    n = 4
    cam = scenes.pinhole_camera(32, 32, cx=16.5, cy=16.5)
    mu = [[0.0, 0.0, z] for z in (2.0, 3.0, 4.0, 5.0)]
    sc = make_scene(mu, np.full((n, 3), math.log(0.05)), [[1, 0, 0, 0]] * n,
                    np.full(n, logit_of(o)), dc_for_colour(np.ones((n, 1, 3))))
    _, _, state = gpu_render(sc, [cam])
    img, T, gid = gpu_images(state)[0]
    # the pixel on the axis: three blends, the fourth Gaussian stops the pixel
    np.testing.assert_allclose(img[16, 16], g["color"][0], rtol=0, atol=2e-6)
    np.testing.assert_allclose(T[16, 16], g["T_final"][0], rtol=2e-5)
    assert gid[16, 16] == int(g["last_contributor"][0])
    p = project(sc, cam)
    tl = tile_lists(p)
    stats = check_view_image(gpu_images(state)[0], p, render_tiles(p, tl=tl), tl)
    assert stats["ambiguous"] == 0
    # gradients of the stack, element by element
    _, grads, g2, gref, acc, p = screen_grads(sc, [cam], 3)
    check_grads({"u": g2[:, 0], "v": g2[:, 1], "opacity": g2[:, 5], "rgb": g2[:, 6:9]},
                acc, ("u", "v", "opacity", "rgb"))
    check_grads({k: to_np(grads[k]) for k in GROUPS}, gref)


def clamp_stack():
    """Four Gaussians far larger than a 24x20 view, at depths 2..5: the front one has
    opacity 0.999, so alpha clamps to 0.99 at every pixel (o G > 0.99 needs m < 0.018,
    i.e. within 0.13 sigma of the mean, and sigma is ~200 pixels); behind it alpha is
    about 0.6, 0.9 and 0.95, so T goes 1 -> 0.01 -> 0.004 -> 0.0004 and the fourth
    would take T below 1e-4: it stops every pixel unblended. The axes differ by up to
    25%, so that the rotations carry a gradient."""
    cam = scenes.pinhole_camera(24, 20)
    f = cam.fy
    zs = (2.0, 3.0, 4.0, 5.0)
    mu = [[0.01 * k, -0.02 * k, z] for k, z in enumerate(zs)]
    # anisotropic, so that the rotations carry a real gradient
    log_s = [[math.log(200.0 * z / f * k) for k in (1.0, 0.8, 1.25)] for z in zs]
    opac = [0.999, 0.6, 0.9, 0.95]
    cols = np.array([[0.9, 0.2, 0.1], [0.1, 0.8, 0.3], [0.3, 0.3, 0.9], [0.7, 0.7, 0.2]])
    q = [[1, 0, 0, 0], [0.9, 0.1, 0.2, 0.1], [0.8, -0.2, 0.1, 0.3], [1, 0, 0, 0]]
    sc = make_scene(mu, log_s, q, logit_of(opac), dc_for_colour(cols[:, None, :]))
    return sc, cam


def test_alpha_clamp_stack_image():
    sc, cam = clamp_stack()
    p = project(sc, cam)
    tl = tile_lists(p)
    ref = render_tiles(p, tl=tl)
    assert np.all(ref.last_id == 2) and not ref.ambiguous_grad.any()
    _, _, state = gpu_render(sc, [cam])
    img, T, gid = gpu_images(state)[0]
    assert np.all(gid == 2)
    check_view_image((img, T, gid), p, ref, tl)


def test_alpha_clamp_stack_gradients():
    sc, cam = clamp_stack()
    _, grads, g2, gref, acc, p = screen_grads(sc, [cam], 4)
    # the clamped front Gaussian: nothing through alpha (mean, whitening, opacity) ...
    assert np.all(g2[0, :6] == 0.0), g2[0]
    assert acc["opacity"][0] == 0.0 and acc["u"][0] == 0.0
    # ... but its colour, and the Gaussians behind it, carry gradient
    assert np.all(np.abs(g2[0, 6:9]) > 0) and np.all(np.abs(g2[1:3, 5]) > 0)
    # the stopped fourth Gaussian gets nothing
    assert np.all(g2[3] == 0.0)
    check_grads({"u": g2[:, 0], "v": g2[:, 1], "opacity": g2[:, 5], "rgb": g2[:, 6:9]},
                acc, ("u", "v", "opacity", "rgb"))
    check_grads({k: to_np(grads[k]) for k in GROUPS}, gref)
    assert to_np(grads["opacity_logits"])[0] == 0.0
