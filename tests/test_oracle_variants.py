"""Pins of the oracle's ablation switches (Sec. 7.3): isotropic Gaussians and
gradients limited to the N front-most Gaussians of each pixel."""
import numpy as np
import pytest

from oracle.adjoint import blend_backward, empty_acc, render_backward
from oracle.gaussians import project
from oracle.raster import render_bruteforce, sort_order
from oracle.rules import Rules
from tests.helpers import make_scene, tiny_random_scene
from tests.test_oracle_adjoint import GROUPS, render_and_fingerprint, with_param


def _equal_rows(sc, rng):
    """The same scene with three equal log-scale rows and random quaternions."""
    ls = np.repeat(sc.log_scales.astype(np.float64).mean(0, keepdims=True), 3, 0)
    q = rng.standard_normal(sc.quats.shape)
    return make_scene(sc.means.T, ls.T, q.T, sc.opacity_logits, sc.sh.transpose(2, 0, 1),
                      sc.sh_degree)


def test_isotropic_equals_anisotropic_with_identity_rotation_and_equal_scales():
    rng = np.random.default_rng(0)
    sc0, cam = tiny_random_scene(6, 10, 1)
    sc = _equal_rows(sc0, rng)
    ident = make_scene(sc.means.T, sc.log_scales.T, np.tile([1.0, 0, 0, 0], (sc.n, 1)),
                       sc.opacity_logits, sc.sh.transpose(2, 0, 1), sc.sh_degree)
    iso = render_bruteforce(project(sc, cam, Rules(isotropic=True)), Rules(isotropic=True))
    ani = render_bruteforce(project(ident, cam, Rules()), Rules())
    np.testing.assert_allclose(iso.color, ani.color, rtol=1e-13, atol=1e-15)
    w = rng.standard_normal((cam.height, cam.width, 3))
    gi, _, _ = render_backward(sc, cam, w, Rules(isotropic=True), bruteforce=True)
    ga, _, _ = render_backward(ident, cam, w, Rules(), bruteforce=True)
    # one radius: each row receives a third of the summed scale gradient; q receives none
    np.testing.assert_allclose(gi["log_scales"], np.repeat(ga["log_scales"].sum(0, keepdims=True) / 3, 3, 0),
                               rtol=1e-12, atol=1e-15)
    assert np.all(gi["quats"] == 0.0)
    for k in ("means", "opacity_logits", "sh"):
        np.testing.assert_allclose(gi[k], ga[k], rtol=1e-12, atol=1e-15)


def test_isotropic_image_ignores_the_quaternion_and_uses_the_mean_log_scale():
    rng = np.random.default_rng(1)
    sc, cam = tiny_random_scene(5, 11, 0)
    r = Rules(isotropic=True)
    a = render_bruteforce(project(sc, cam, r), r).color
    sc2 = make_scene(sc.means.T, sc.log_scales.T[:, ::-1], rng.standard_normal((sc.n, 4)),
                     sc.opacity_logits, sc.sh.transpose(2, 0, 1), sc.sh_degree)
    b = render_bruteforce(project(sc2, cam, r), r).color
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)
    p = project(sc, cam, Rules(isotropic=True))
    s = np.exp(sc.log_scales.astype(np.float64).mean(0))
    np.testing.assert_allclose(p.Sigma, s[:, None, None] ** 2 * np.eye(3), rtol=1e-13, atol=1e-300)


def test_isotropic_gradient_matches_central_differences():
    rules = Rules(isotropic=True)
    sc, cam = tiny_random_scene(6, 12, 2)
    w = np.random.default_rng(13).standard_normal((cam.height, cam.width, 3))
    g, _, _ = render_backward(sc, cam, w, rules, bruteforce=True)
    _, fp0 = render_and_fingerprint(sc, cam, rules)
    checked = 0
    for group in ("means", "log_scales", "quats"):
        base = getattr(sc, group).astype(np.float64)
        scale = np.abs(g[group]).max() + 1e-12
        for index in np.ndindex(base.shape):
            th = base[index]
            h = 1e-6 * max(1.0, abs(th))
            cp, fpp = render_and_fingerprint(with_param(sc, group, index, th + h), cam, rules)
            cm, fpm = render_and_fingerprint(with_param(sc, group, index, th - h), cam, rules)
            if fpp != fp0 or fpm != fp0:
                continue
            fd = ((w * cp).sum() - (w * cm).sum()) / (2 * h)
            assert abs(fd - g[group][index]) <= 2e-6 * (abs(fd) + scale), (group, index)
            checked += 1
    assert checked >= 40


def _per_pixel_unlimited(sc, cam, w):
    """Screen-space gradients of each pixel alone (unlimited), and the front-to-back
    rank of every (pixel, Gaussian) blend, by brute force over single pixels."""
    rules = Rules()
    p = project(sc, cam, rules)
    ids = sort_order(p, p.drawable)
    H, W = cam.height, cam.width
    per, ranks = [], []
    for j in range(H):
        for i in range(W):
            acc = empty_acc(p.n)
            fwd = blend_backward(p, ids, np.array([i]), np.array([j]), w[j, i][None], rules, acc)
            order = [st[1] for st in fwd.steps if st[2][0]]
            per.append(acc)
            ranks.append({g: r for r, g in enumerate(order)})
    return p, per, ranks


@pytest.mark.parametrize("N", [1, 2, 3])
def test_limited_gradient_is_the_front_most_part_of_each_pixels_gradient(N):
    sc, cam = tiny_random_scene(7, 14, 1, width=12, height=10, spread=0.3,
                                log_s=(np.log(0.35), 0.2))
    w = np.random.default_rng(15).standard_normal((cam.height, cam.width, 3))
    p, per, ranks = _per_pixel_unlimited(sc, cam, w)
    want = empty_acc(p.n)
    for acc, rk in zip(per, ranks):
        for g, r in rk.items():
            if r < N:
                for k in want:
                    want[k][g] += acc[k][g]
    _, got, _ = render_backward(sc, cam, w, Rules(grad_limit=N), bruteforce=True)
    assert max(len(r) for r in ranks) > N      # the limit removes something
    for k in want:
        np.testing.assert_allclose(got[k], want[k], rtol=1e-12, atol=1e-15)


def test_limit_above_every_depth_complexity_is_the_full_gradient():
    sc, cam = tiny_random_scene(6, 16, 1)
    w = np.random.default_rng(17).standard_normal((cam.height, cam.width, 3))
    full, _, _ = render_backward(sc, cam, w, Rules(), bruteforce=True)
    lim, _, _ = render_backward(sc, cam, w, Rules(grad_limit=6), bruteforce=True)
    for k in GROUPS:
        np.testing.assert_array_equal(lim[k], full[k])
