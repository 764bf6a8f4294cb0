"""Pins of the oracle's decision margins and alternative outcomes (App. C thresholds).

* A hand-derived case at a threshold: two Gaussians clamped at alpha = 0.99 on one
  pixel centre give T' = (1 - 0.99)^2, which is 1e-4 up to FP64 rounding. Such a
  decision must be flagged, and the two legitimate outcomes are known by hand:
  both blended (colour 0.99 + 0.01 * 0.99 = 0.9999, T = 1e-4) or the second one
  stopping the pixel (colour 0.99, T = 0.01).
* The FP32 error model: the same blend evaluated in IEEE binary32 (NumPy float32
  from FP32-rounded inputs, the mean relative to its box corner, the whitened
  inverse covariance) must take every decision the FP64 oracle takes except where
  the oracle flags the pixel, and its final transmittance must lie within the
  oracle's bound T_err.
"""
import math

import numpy as np
import pytest

import scenes
from oracle.gaussians import project
from oracle.raster import (DECIDE_STOP, blend, pixel_outcomes, render_tiles, tile_lists,
                           tile_pixels)
from tests.helpers import dc_for_colour, logit_of, make_scene


def test_outcomes_at_the_stop_threshold():
    cam = scenes.pinhole_camera(32, 32, cx=16.5, cy=16.5)
    mu = [[0.0, 0.0, 2.0], [0.0, 0.0, 3.0]]
    sc = make_scene(mu, np.full((2, 3), math.log(0.2)), [[1, 0, 0, 0]] * 2,
                    np.full(2, logit_of(0.999999)), dc_for_colour(np.ones((2, 1, 3))))
    p = project(sc, cam)
    tl = tile_lists(p)
    t = (16 // 16) * tl.tiles_x + 16 // 16
    ids = tl.ids[tl.start[t]:tl.start[t + 1]]
    base = blend(p, ids, np.array([16]), np.array([16]), flags=True)
    assert base.ambiguous[0]
    assert base.flags[0] == [(1, DECIDE_STOP)]
    outs = pixel_outcomes(p, ids, 16, 16)
    assert len(outs) == 2
    got = sorted((float(o.color[0, 0]), float(o.T_final[0]), int(o.last_id[0])) for o in outs)
    np.testing.assert_allclose(got[0][:2], [0.99, 0.01], rtol=1e-12)
    assert got[0][2] == 0
    np.testing.assert_allclose(got[1][:2], [0.9999, 1e-4], rtol=1e-12)
    assert got[1][2] == 1


def test_forcing_nothing_is_the_plain_blend():
    sc = scenes.uniform_scene(300, 5, 1, (2.0, 6.0))
    cam = scenes.pinhole_camera(48, 40)
    p = project(sc, cam)
    tl = tile_lists(p)
    for t in range(tl.tiles_x * tl.tiles_y):
        px, py = tile_pixels(t, tl, cam.width, cam.height, 16)
        ids = tl.ids[tl.start[t]:tl.start[t + 1]]
        a = blend(p, ids, px, py)
        b = blend(p, ids, px, py, flags=True)
        np.testing.assert_array_equal(a.color, b.color)
        np.testing.assert_array_equal(a.T_final, b.T_final)
        assert all(bool(f) == bool(x) for f, x in zip(b.flags, b.ambiguous))


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def _fma32(a, b, c):
    # a * b + c with one rounding (the FP64 product of two binary32 values is exact)
    return _f32(a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64))


def fp32_blend(p, ids, px, py):
    """The blend of the same list in IEEE binary32 from FP32-rounded per-Gaussian inputs:
    m = |W D + c|^2 with W the whitening factor, D the pixel's offset from the centre of
    the box's corner pixel and c the whitened offset of that centre from the mean."""
    P = px.size
    T = np.ones(P, np.float32)
    last = np.full(P, -1, np.int64)
    live = np.ones(P, bool)
    a_min, a_max, t_min = np.float32(1 / 255), np.float32(0.99), np.float32(1e-4)
    for g in ids:
        a, b, c = p.cov2d[g, 0, 0], p.cov2d[g, 0, 1], p.cov2d[g, 1, 1]
        l00 = math.sqrt(a)
        l10 = b / l00
        l11 = math.sqrt(c - l10 * l10)
        w00, w10, w11 = 1 / l00, -l10 / (l00 * l11), 1 / l11
        ax, ay = (p.i_lo[g] + 0.5) - p.u[g], (p.j_lo[g] + 0.5) - p.v[g]
        c0, c1 = _f32(w00 * ax), _f32(w10 * ax + w11 * ay)
        w00, w10, w11 = _f32(w00), _f32(w10), _f32(w11)
        Di = (px - p.i_lo[g]).astype(np.float32)
        Dj = (py - p.j_lo[g]).astype(np.float32)
        e0 = _fma32(np.broadcast_to(w00, Di.shape), Di, np.broadcast_to(c0, Di.shape))
        inner = _fma32(np.broadcast_to(w11, Dj.shape), Dj, np.broadcast_to(c1, Dj.shape))
        e1 = _fma32(np.broadcast_to(w10, Di.shape), Di, inner)
        m = _fma32(e0, e0, e1 * e1)
        G = np.exp(np.float32(-0.5) * m)
        alpha = np.minimum(a_max, _f32(p.opacity[g]) * G)
        take = live & (m <= np.float32(9.0)) & (alpha >= a_min)
        Tn = T * (np.float32(1.0) - alpha)
        stop = take & (Tn < t_min)
        blended = take & ~stop
        T = np.where(blended, Tn, T)
        last = np.where(blended, g, last)
        live &= ~stop
    return T.astype(np.float64), last


@pytest.mark.parametrize("name,seed", [("small", 0), ("dense", 1), ("thin", 2)])
def test_fp32_evaluation_flips_only_flagged_decisions_and_stays_in_the_T_bound(name, seed):
    if name == "small":
        sc, cams = scenes.workload("small")
        cam = cams[0]
    elif name == "dense":
        # many opaque Gaussians: long lists, most pixels stop on the T rule
        sc = scenes.uniform_scene(3000, seed, 0, (2.0, 6.0))
        sc.opacity_logits[:] = np.abs(sc.opacity_logits) + 1.0
        cam = scenes.pinhole_camera(64, 48)
    else:
        # needle-like Gaussians (axis ratios up to 100:1) near their extent
        sc = scenes.uniform_scene(800, seed, 0, (2.0, 6.0))
        sc.log_scales[0] += 2.5
        sc.log_scales[1] -= 2.0
        cam = scenes.pinhole_camera(64, 48)
    p = project(sc, cam)
    tl = tile_lists(p)
    ref = render_tiles(p, tl=tl)
    n_checked = 0
    for t in range(tl.tiles_x * tl.tiles_y):
        px, py = tile_pixels(t, tl, cam.width, cam.height, 16)
        ids = tl.ids[tl.start[t]:tl.start[t + 1]]
        T32, last32 = fp32_blend(p, ids, px, py)
        amb = ref.ambiguous[py, px]
        same = last32 == ref.last_id[py, px]
        assert np.all(same | amb), (t, np.nonzero(~same & ~amb))
        ok = ~amb
        T64, err = ref.T_final[py, px][ok], ref.T_err[py, px][ok]
        assert np.all(np.abs(T32[ok] - T64) <= T64 * (err + 2.0 ** -24)), t
        n_checked += int(ok.sum())
    assert n_checked > 0.99 * cam.width * cam.height


def threshold_scenes():
    """Scenes whose exact decisions sit on a threshold at some pixel centres."""
    cam = scenes.pinhole_camera(32, 32, cx=16.5, cy=16.5)
    f = cam.fx
    out = []
    # T' = (1 - 0.99)^2: 1e-4 in FP64 up to rounding, below it in FP32
    out.append(make_scene([[0.0, 0.0, 2.0], [0.0, 0.0, 3.0]], np.full((2, 3), math.log(0.2)),
                          [[1, 0, 0, 0]] * 2, np.full(2, logit_of(0.999999)),
                          dc_for_colour(np.ones((2, 1, 3)))))
    # isotropic Gaussians whose 3-sigma circle passes through pixel centres (m = 9 at
    # offsets (3, 0), (0, 3), and at (5, 0) for sigma = 5/3 px)
    zs = np.array([2.0, 2.5, 3.0, 3.5])
    sig_px = np.array([1.0, 5.0 / 3.0, 1.0, 5.0 / 3.0])
    out.append(make_scene(np.stack([np.zeros(4), np.zeros(4), zs], 1),
                          np.repeat(np.log(sig_px * zs / f)[:, None], 3, 1), [[1, 0, 0, 0]] * 4,
                          np.full(4, logit_of(0.5)), dc_for_colour(np.full((4, 1, 3), 0.7))))
    # alpha = 1/255 exactly at one pixel centre: o exp(-m/2) = 1/255 at m = 4
    o = math.exp(2.0) / 255.0
    out.append(make_scene([[0.0, 0.0, 3.0]], np.full((1, 3), math.log(1.0 * 3.0 / f)),
                          [[1, 0, 0, 0]], [logit_of(o)], dc_for_colour(np.ones((1, 1, 3)))))
    return cam, out


def test_fp32_flips_are_flagged_and_among_the_outcomes():
    cam, cases = threshold_scenes()
    flips = 0
    for sc in cases:
        p = project(sc, cam)
        tl = tile_lists(p)
        ref = render_tiles(p, tl=tl)
        for t in range(tl.tiles_x * tl.tiles_y):
            px, py = tile_pixels(t, tl, cam.width, cam.height, 16)
            ids = tl.ids[tl.start[t]:tl.start[t + 1]]
            T32, last32 = fp32_blend(p, ids, px, py)
            for k in np.nonzero(last32 != ref.last_id[py, px])[0]:
                x, y = int(px[k]), int(py[k])
                assert ref.ambiguous[y, x], (x, y)
                outs = pixel_outcomes(p, ids, x, y)
                assert any(o.last_id[0] == last32[k] and
                           abs(o.T_final[0] - T32[k]) <= o.T_final[0] * (o.T_err[0] + 2.0 ** -24)
                           for o in outs), (x, y)
                flips += 1
    assert flips >= 1
