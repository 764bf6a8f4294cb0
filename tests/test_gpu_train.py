"""Adam, the densification gather and the training loop on the GPU."""
import numpy as np
import pytest

import scenes
from oracle import density as od
from oracle import optim as oo
from tests.gpu_common import GROUPS, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("offset", [0, 1])
def test_adam_step_matches_oracle(offset):
    import torch
    from paper_2308_04079_amd import _lib
    rng = np.random.default_rng(offset)
    n = 10_003
    p0 = rng.standard_normal(n + offset).astype(np.float32)
    P = torch.from_numpy(p0).cuda()
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    p, m, v = p0[offset:].astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = rng.standard_normal(n + offset).astype(np.float32)
        G = torch.from_numpy(g).cuda()
        # offset 1 gives arrays that are not 16-byte aligned (the scalar path)
        _lib.check("gs_adam_step", _lib.lib().gs_adam_step(
            _lib.ptr(P) + 4 * offset, _lib.ptr(G) + 4 * offset, _lib.ptr(M) + 4 * offset,
            _lib.ptr(V) + 4 * offset, n, 1e-2, 0.9, 0.999, 1e-8, t, None))
        p, m, v = oo.adam_step(p, g[offset:].astype(np.float64), m, v, t, 1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(to_np(P)[offset:], p, rtol=2e-5, atol=2e-6)
    np.testing.assert_allclose(to_np(M)[offset:], m, rtol=2e-5, atol=1e-7)
    if offset:
        assert to_np(P)[0] == p0[0]          # nothing outside the range is touched


def test_gather_carries_kept_state_and_zeroes_created():
    import ctypes

    import torch
    from paper_2308_04079_amd import GaussianParams, _lib
    from paper_2308_04079_amd.density import DensityControl
    sc = scenes.uniform_scene(5000 + 7, 3, sh_degree=2)
    rng = np.random.default_rng(4)
    dc = DensityControl(sc.n, split_scale=0.05)
    dc.grad_sum.copy_(torch.from_numpy((rng.random(sc.n) * 1e-3).astype(np.float32)))
    dc.view_count.copy_(torch.from_numpy(rng.integers(0, 3, sc.n).astype(np.int32)))
    params = GaussianParams.from_numpy(sc)
    action, offsets, n_new = dc.plan(params)
    state = GaussianParams(*(torch.randn_like(getattr(params, k)) for k in GROUPS))
    for zero in (0, 1):
        out = GaussianParams(torch.empty(3, n_new, device="cuda"), torch.empty(3, n_new, device="cuda"),
                             torch.empty(4, n_new, device="cuda"), torch.empty(n_new, device="cuda"),
                             torch.empty(9, 3, n_new, device="cuda"))
        dst = _lib.GsParamsGrad(*(_lib.ptr(getattr(out, k)) for k in GROUPS))
        _lib.check("gs_densify_gather", _lib.lib().gs_densify_gather(
            ctypes.byref(state.c_struct()), 2, _lib.ptr(action), _lib.ptr(offsets), zero,
            ctypes.byref(dst), n_new, None))
        torch.cuda.synchronize()
        act = to_np(action).astype(np.int64)
        src = np.repeat(np.arange(sc.n), np.array([0, 1, 2, 2])[act])
        keep = (act[src] == od.KEEP) | (zero == 0)
        assert len(src) == n_new
        for k in GROUPS:
            a = to_np(getattr(state, k))
            b = to_np(getattr(out, k))
            np.testing.assert_array_equal(b, a[..., src] * keep)


def test_training_loop_reduces_the_loss_and_densifies():
    import torch
    from paper_2308_04079_amd import GaussianParams, Rasterizer
    from paper_2308_04079_amd.train import TrainConfig, Trainer
    torch.manual_seed(0)
    target_sc = scenes.uniform_scene(3000, 31, sh_degree=3)
    start = scenes.jitter_means(target_sc, 32, sd=0.05)
    start.opacity_logits[:] = 0.0
    start.log_scales[:] += 0.3
    cams = [scenes.look_at_camera([0.3 * np.cos(a), 0.2 * np.sin(a), -0.5], [0, 0, 4.0], 160, 120)
            for a in np.linspace(0, 2 * np.pi, 6, endpoint=False)]
    r = Rasterizer(sh_degree=3)
    tparams = GaussianParams.from_numpy(target_sc)
    targets = [r.render(tparams, [c]).image.clone() for c in cams]
    cfg = TrainConfig(iterations=300, views_per_step=2, warmup=(20, 40), sh_every=40,
                      densify_from=60, densify_until=220, densify_every=40, reset_every=150,
                      lr_means=(1.6e-4, 1.6e-6))
    tr = Trainer(GaussianParams.from_numpy(start), cams, targets, extent=2.0, cfg=cfg)
    counts = []
    for _ in range(cfg.iterations):
        tr.step()
        counts.append(tr.params.n)
    losses = torch.stack([x.sum() for x in tr.history]).cpu().numpy()
    assert np.isfinite(losses).all()
    assert losses[280:].mean() < 0.8 * losses[40:60].mean(), (losses[40:60].mean(), losses[280:].mean())
    assert len(set(counts)) > 1                         # density control changed the model
    assert tr.m.means.shape == tr.params.means.shape
    assert tr.sh_degree(tr.it) == 3


def test_sh_bands_before_the_ramp_stay_untouched():
    """Bands the SH ramp has not reached get no update and keep zero moments (the
    Adam step on them is skipped, which equals running it on zero gradients)."""
    import torch
    from paper_2308_04079_amd import GaussianParams, Rasterizer
    from paper_2308_04079_amd.train import TrainConfig, Trainer
    sc = scenes.uniform_scene(2000, 35, sh_degree=3)
    cams = [scenes.look_at_camera([0.2 * np.cos(a), 0.1, -0.5], [0, 0, 4.0], 96, 72)
            for a in np.linspace(0, 2 * np.pi, 3, endpoint=False)]
    r = Rasterizer(sh_degree=3)
    tgt = GaussianParams.from_numpy(scenes.jitter_means(sc, 36, sd=0.05))
    targets = [r.render(tgt, [c]).image.clone() for c in cams]
    cfg = TrainConfig(iterations=30, views_per_step=1, warmup=(0, 0), sh_every=10,
                      densify_from=1000, densify_until=999, reset_every=10 ** 6)
    tr = Trainer(GaussianParams.from_numpy(sc), cams, targets, extent=2.0, cfg=cfg)
    sh0 = tr.params.sh.clone()
    for _ in range(15):                                   # degree 0 for 10 steps, then 1
        tr.step()
    torch.cuda.synchronize()
    assert torch.equal(tr.params.sh[4:], sh0[4:])         # degrees 2 and 3 not reached
    assert not torch.any(tr.m.sh[4:]) and not torch.any(tr.v.sh[4:])
    assert not torch.equal(tr.params.sh[1:4], sh0[1:4])   # degree 1 active for 5 steps
    assert not torch.equal(tr.params.sh[0], sh0[0])
