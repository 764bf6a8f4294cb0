"""Pins of the oracle's photometric loss (Sec. 5.1: L1 and D-SSIM)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import loss as ol


def test_window_is_the_normalised_sampled_gaussian():
    w = ol.gaussian_window()
    assert w.shape == (11, 11)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(w, w.T, rtol=0, atol=0)
    g = w.sum(1)
    np.testing.assert_allclose(g[5] / g[4], np.exp(1.0 / (2 * 1.5 ** 2)), rtol=1e-14)
    np.testing.assert_allclose(g[4] / g[3], np.exp(3.0 / (2 * 1.5 ** 2)), rtol=1e-14)


def test_window_sum_is_scipys_gaussian_filter_with_zero_borders():
    # a library routine: radius int(truncate * sigma + 0.5) = 5, zero outside the image
    x = np.random.default_rng(0).random((2, 23, 17))
    ref = np.stack([ndimage.gaussian_filter(c, 1.5, mode="constant", cval=0.0, truncate=5 / 1.5)
                    for c in x])
    np.testing.assert_allclose(ol.window_filter(x, ol.gaussian_window()), ref, rtol=1e-13, atol=1e-15)


def _ssim_at(x, y, i, j):
    """SSIM of one pixel straight from the definition, by explicit sums."""
    w = ol.gaussian_window()
    H, W = x.shape
    s = dict(mx=0.0, my=0.0, xx=0.0, yy=0.0, xy=0.0)
    for a in range(-5, 6):
        for b in range(-5, 6):
            if 0 <= i + a < H and 0 <= j + b < W:
                wt = w[a + 5, b + 5]
                u, v = x[i + a, j + b], y[i + a, j + b]
                s["mx"] += wt * u
                s["my"] += wt * v
                s["xx"] += wt * u * u
                s["yy"] += wt * v * v
                s["xy"] += wt * u * v
    vx = s["xx"] - s["mx"] ** 2
    vy = s["yy"] - s["my"] ** 2
    cv = s["xy"] - s["mx"] * s["my"]
    return ((2 * s["mx"] * s["my"] + ol.C1) * (2 * cv + ol.C2)) / (
        (s["mx"] ** 2 + s["my"] ** 2 + ol.C1) * (vx + vy + ol.C2))


def test_ssim_map_against_the_definition_at_corners_edges_and_interior():
    rng = np.random.default_rng(1)
    x, y = rng.random((14, 19)), rng.random((14, 19))
    S = ol.ssim_terms(x, y)["ssim"]
    for i, j in [(0, 0), (0, 18), (13, 0), (13, 18), (3, 9), (7, 7), (13, 4), (6, 0)]:
        assert abs(S[i, j] - _ssim_at(x, y, i, j)) < 1e-12


def test_ssim_of_constant_images_in_the_interior():
    a, b = 0.3, 0.7
    x, y = np.full((1, 21, 21), a), np.full((1, 21, 21), b)
    S = ol.ssim_terms(x, y)["ssim"][0]
    closed = (2 * a * b + ol.C1) / (a * a + b * b + ol.C1)
    np.testing.assert_allclose(S[5:-5, 5:-5], closed, rtol=1e-12)
    # at the border the zero padding is part of the window: not the closed form
    assert abs(S[0, 0] - closed) > 1e-3


def test_identical_images_give_zero_loss_and_zero_gradient():
    x = np.random.default_rng(2).random((3, 12, 15))
    loss, g = ol.dssim(x, x)
    assert abs(loss) < 1e-14
    assert np.abs(g).max() < 1e-12
    S = ol.ssim_terms(x, 1.0 - x)["ssim"]
    assert (S <= 1.0).all() and (S >= -1.0).all()
    np.testing.assert_allclose(ol.ssim_terms(1.0 - x, x)["ssim"], S, rtol=1e-12)


@pytest.mark.parametrize("fn", [ol.dssim, ol.photometric])
def test_gradient_against_central_differences(fn):
    rng = np.random.default_rng(3)
    x, y = rng.random((3, 9, 13)), rng.random((3, 9, 13))
    loss, g = fn(x, y)
    h = 1e-6
    idx = [(0, 0, 0), (1, 4, 6), (2, 8, 12), (0, 8, 1), (2, 3, 11), (1, 0, 7)]
    for k in idx:
        xp, xm = x.copy(), x.copy()
        xp[k] += h
        xm[k] -= h
        fd = (fn(xp, y)[0] - fn(xm, y)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_l1_value_and_gradient():
    x = np.array([[[0.2, 0.5], [0.9, 0.4]]])
    y = np.array([[[0.1, 0.5], [1.0, 0.0]]])
    loss, g = ol.l1(x, y)
    assert abs(loss - (0.1 + 0.0 + 0.1 + 0.4) / 4) < 1e-15
    np.testing.assert_array_equal(g, np.array([[[1, 0], [-1, 1]]]) / 4)
