"""Pins of the oracle's Adam step and schedule."""
import math

import numpy as np
import torch

from oracle import optim as oo


def test_first_adam_step_moves_by_lr_times_sign():
    # with zero moments, m_hat = g and v_hat = g^2 after bias correction
    g = np.array([3.0, -0.5, 1e-3])
    p, m, v = oo.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-12)


def test_adam_equals_torch_adam_on_the_cpu():
    rng = np.random.default_rng(0)
    p0 = rng.standard_normal(50)
    x = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([x], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        g = rng.standard_normal(50)
        x.grad = torch.tensor(g)
        opt.step()
        p, m, v = oo.adam_step(p, g, m, v, t, 3e-3)
    np.testing.assert_allclose(p, x.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_schedule():
    assert math.isclose(oo.position_lr(0, 100, 1e-3, 1e-5), 1e-3, rel_tol=1e-12)
    assert math.isclose(oo.position_lr(50, 100, 1e-3, 1e-5), 1e-4, rel_tol=1e-12)
    assert math.isclose(oo.position_lr(200, 100, 1e-3, 1e-5), 1e-5, rel_tol=1e-12)
    assert [oo.resolution_divisor(i) for i in (0, 249, 250, 499, 500)] == [4, 4, 2, 2, 1]
    assert [oo.sh_degree_at(i) for i in (0, 999, 1000, 2500, 3000, 9000)] == [0, 0, 1, 2, 3, 3]
    assert [oo.densify_now(i) for i in (100, 400, 500, 550, 600, 15000, 15100)] == \
        [False, False, True, False, True, True, False]
    assert [oo.reset_opacity_now(i) for i in (0, 2999, 3000, 6000)] == [False, False, True, True]
