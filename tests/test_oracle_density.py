"""Pins of the oracle's adaptive density control (Sec. 5.2, Alg. 1)."""
import math

import numpy as np

from oracle.density import (CLONE, KEEP, REMOVE, SPLIT, DensifyRules, accumulate, apply, plan,
                            reset_opacity)
from oracle.gaussians import quaternion_to_rotation
from tests.helpers import make_scene


def scene_with(logits, log_scales):
    n = len(logits)
    return make_scene(np.zeros((n, 3)), log_scales, np.tile([1.0, 0.2, -0.3, 0.5], (n, 1)),
                      logits, np.arange(n * 3, dtype=float).reshape(n, 1, 3))


def test_ndc_gradient_norm():
    # du = 1 per pixel on a 100-wide image is 50 per NDC unit; dv = 1 on 40 rows is 20
    s, c = accumulate([[1.0, 0.0]], [[0.0, 1.0]], np.array([[True, True]]), [100], [40])
    np.testing.assert_allclose(s, [50.0, 20.0])
    s, c = accumulate([[3.0], [4.0]], [[0.0], [0.0]], np.array([[True], [False]]), [2, 2], [2, 2])
    assert s[0] == 3.0 and c[0] == 1


def test_plan_follows_algorithm_1():
    r = DensifyRules(grad_threshold=0.0002, min_opacity=0.005, split_scale=0.05)
    lg = [math.log(0.001 / 0.999), 0.0, 0.0, 0.0, 0.0]
    ls = [[-3, -3, -3], [-4, -4, -4], [-4, -4, -4], [-1, -4, -4], [-4, -4, -4]]
    sc = scene_with(lg, ls)
    grad_sum = np.array([1.0, 0.0, 0.001, 0.001, 0.0003])
    count = np.array([1, 1, 2, 2, 2])
    act, cnt = plan(sc, grad_sum, count, np.zeros(5), r)
    # transparent removed; no gradient kept; small densified cloned; large split;
    # average 0.00015 < tau kept
    assert act.tolist() == [REMOVE, KEEP, CLONE, SPLIT, KEEP]
    assert cnt.tolist() == [0, 1, 2, 2, 1]


def test_apply_clone_copies_and_split_samples_the_gaussian():
    r = DensifyRules()
    sc = scene_with([0.0, 0.0, 0.0], [[-2, -1, -3], [-1, -2, -0.5], [-2, -2, -2]])
    act = np.array([KEEP, CLONE, SPLIT])
    z = np.random.default_rng(0).standard_normal((3, 2, 3))
    out = apply(sc, act, z, r)
    assert out["src"].tolist() == [0, 1, 1, 2, 2]
    np.testing.assert_array_equal(out["means"][1], out["means"][2])
    np.testing.assert_allclose(out["log_scales"][3], sc.log_scales[:, 2] - math.log(1.6))
    np.testing.assert_array_equal(out["sh"][4], sc.sh[:, :, 2])


def test_split_children_are_distributed_as_the_parent():
    # children positions sampled with the parent as the PDF: covariance R S^2 R^T
    rng = np.random.default_rng(1)
    ls = np.array([[-1.0, -2.0, -0.5]])
    q = np.array([[0.8, 0.3, -0.2, 0.4]])
    sc = make_scene([[1.0, 2.0, 3.0]], ls, q, [0.0], np.zeros((1, 1, 3)))
    m = 20000
    pos = np.concatenate([apply(sc, np.array([SPLIT]), rng.standard_normal((1, 2, 3)))["means"]
                          for _ in range(m // 2)])
    Rq = quaternion_to_rotation(q / np.linalg.norm(q))[0]
    Sigma = Rq @ np.diag(np.exp(2 * ls[0])) @ Rq.T
    np.testing.assert_allclose(pos.mean(0), [1, 2, 3], atol=4 * math.sqrt(Sigma.max() / m))
    np.testing.assert_allclose(np.cov(pos.T), Sigma, atol=0.05 * np.abs(Sigma).max())


def test_opacity_reset_caps_alpha():
    lg = reset_opacity([5.0, -10.0, 0.0], 0.01)
    o = 1 / (1 + np.exp(-lg))
    np.testing.assert_allclose(o, [0.01, 1 / (1 + math.exp(10)), 0.01], rtol=1e-12)


def test_removal_by_size():
    sc = scene_with([0.0, 0.0], [[0.0, -3, -3], [-3, -3, -3]])
    act, _ = plan(sc, np.zeros(2), np.zeros(2, int), np.array([1.0, 50.0]),
                  DensifyRules(max_world_scale=0.5, max_screen_radius=20.0))
    assert act.tolist() == [REMOVE, REMOVE]
