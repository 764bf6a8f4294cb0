"""The training driver's schedule against the oracle's (CPU)."""
import math

from oracle import optim as oo
from paper_2308_04079_amd.train import TrainConfig, Trainer


def test_trainer_schedule_equals_oracle_schedule():
    t = object.__new__(Trainer)
    t.cfg = TrainConfig()
    t.extent = 2.5
    t.max_deg = 3
    for it in list(range(0, 1200, 7)) + [2999, 3000, 3001, 6000, 14999, 15000, 15100, 29999, 30000]:
        assert t.resolution_divisor(it) == oo.resolution_divisor(it)
        assert t.sh_degree(it) == oo.sh_degree_at(it)
        assert t.densify_now(it) == oo.densify_now(it), it
        assert t.reset_now(it) == oo.reset_opacity_now(it)
        assert math.isclose(t.lr_means(it), 2.5 * oo.position_lr(it, 30000, 1.6e-4, 1.6e-6),
                            rel_tol=1e-12)


def test_warmup_targets_and_cameras():
    """The warm-up renders at 1/div resolution: the camera keeps every pixel centre's
    ray (pixel centre (i + 0.5) div of the full view maps to (i + 0.5) of the small
    one), and the target is the div x div box mean of the full image."""
    import types

    import numpy as np
    import torch
    from paper_2308_04079_amd.train import downsample, scaled_camera
    cam = types.SimpleNamespace(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32),
                                fx=np.float32(800.0), fy=np.float32(790.0),
                                cx=np.float32(321.0), cy=np.float32(239.0), width=643, height=481)
    for div in (1, 2, 4):
        small = scaled_camera(cam, div)
        assert (small.width, small.height) == (643 // div, 481 // div)
        # the ray through small pixel centre (i + 0.5) is the full view's through (i + 0.5) div
        for i in (0.5, 10.5, small.width - 0.5):
            x_small = (i - float(small.cx)) / float(small.fx)
            x_full = (i * div - float(cam.cx)) / float(cam.fx)
            assert math.isclose(x_small, x_full, rel_tol=1e-6, abs_tol=1e-6)
        img = torch.rand(3, 481, 643, dtype=torch.float64)
        d = downsample(img, cam, div).view(3, 481 // div, 643 // div)
        h, w = 481 // div, 643 // div
        ref = img[:, :h * div, :w * div].numpy().reshape(3, h, div, w, div).mean(axis=(2, 4))
        np.testing.assert_allclose(d.numpy(), ref, rtol=1e-12)
