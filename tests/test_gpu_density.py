"""Adaptive density control on the GPU against the oracle (Sec. 5.2, Alg. 1)."""
import numpy as np
import pytest

import scenes
from oracle import density as od
from tests.gpu_common import GROUPS, to_np

pytestmark = pytest.mark.gpu


def _clear_of(x, thresholds, rel=1e-4):
    """Push values away from every decision threshold (both sides decide alike)."""
    x = np.array(x, dtype=np.float64)
    for _ in range(20):
        near = np.zeros(x.shape, bool)
        for t in thresholds:
            near |= np.abs(x - t) <= rel * abs(t)
        if not near.any():
            break
        x[near] *= 1.0 + 10 * rel
    return x


def _synthetic_stats(n, seed, rules):
    rng = np.random.default_rng(seed)
    sc = scenes.uniform_scene(n, seed, sh_degree=1)
    # opacities around epsilon_alpha, scales around the split and size thresholds
    o = np.exp(rng.uniform(np.log(1e-3), np.log(0.9), n))
    o = _clear_of(o, [rules.min_opacity])
    sc.opacity_logits[:] = np.log(o / (1 - o)).astype(np.float32)
    ls = rng.normal(np.log(rules.split_scale), 1.0, (3, n))
    smax = _clear_of(np.exp(ls.max(0)), [rules.split_scale, rules.max_world_scale])
    ls[ls.argmax(0), np.arange(n)] = np.log(smax)
    sc.log_scales[:] = ls.astype(np.float32)
    # recompute from the FP32 values both sides read
    count = rng.integers(0, 6, n).astype(np.int32)
    avg = _clear_of(np.exp(rng.uniform(np.log(2e-5), np.log(2e-3), n)), [rules.grad_threshold])
    grad_sum = (avg * count).astype(np.float32)
    radius = _clear_of(rng.uniform(0.5, 80, n).round() / 2, [rules.max_screen_radius]).astype(np.float32)
    return sc, grad_sum, count, radius


def _rules_pair(**kw):
    from paper_2308_04079_amd.density import DensityControl
    return od.DensifyRules(**kw), kw, DensityControl


@pytest.mark.parametrize("kw", [{}, {"max_world_scale": 0.05, "max_screen_radius": 20.0,
                                     "split_scale": 0.02}])
def test_plan_and_offsets_match_oracle(kw):
    import torch
    from paper_2308_04079_amd import GaussianParams
    rules, kw, DC = _rules_pair(**kw)
    n = 20000 + 777    # several scan blocks and a ragged tail
    sc, gsum, cnt, rad = _synthetic_stats(n, 5, rules)
    # the oracle reads the same FP32 values (an FP32 average of the FP32 sum decides)
    act_o, out_o = od.plan(sc, gsum.astype(np.float64), cnt, rad.astype(np.float64), rules)
    dc = DC(n, **kw)
    dc.grad_sum.copy_(torch.from_numpy(gsum))
    dc.view_count.copy_(torch.from_numpy(cnt))
    dc.max_radius.copy_(torch.from_numpy(rad))
    params = GaussianParams.from_numpy(sc)
    action, offsets, n_new = dc.plan(params)
    act_g = to_np(action).astype(np.int64)
    np.testing.assert_array_equal(act_g, act_o)
    assert n_new == int(out_o.sum())
    np.testing.assert_array_equal(to_np(offsets).astype(np.int64), np.cumsum(out_o) - out_o)
    assert set(act_o.tolist()) == {od.REMOVE, od.KEEP, od.CLONE, od.SPLIT}


def test_apply_matches_oracle():
    import torch
    from paper_2308_04079_amd import GaussianParams
    rules, kw, DC = _rules_pair()
    n = 5000 + 13
    sc, gsum, cnt, rad = _synthetic_stats(n, 7, rules)
    act_o, out_o = od.plan(sc, gsum.astype(np.float64), cnt, rad.astype(np.float64), rules)
    z = np.random.default_rng(8).standard_normal((n, 2, 3)).astype(np.float32)
    ref = od.apply(sc, act_o, z.astype(np.float64), rules)
    dc = DC(n)
    dc.grad_sum.copy_(torch.from_numpy(gsum))
    dc.view_count.copy_(torch.from_numpy(cnt))
    params = GaussianParams.from_numpy(sc)
    action, offsets, n_new = dc.plan(params)
    out, src = dc.apply(params, action, offsets, n_new, torch.from_numpy(z).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(src), ref["src"])
    split = act_o[ref["src"]] == od.SPLIT
    for k in GROUPS:
        got = to_np(getattr(out, k)).astype(np.float64)
        got = got.reshape(-1, got.shape[-1]).T if k != "opacity_logits" else got
        exp = ref[k].reshape(len(ref["src"]), -1)
        got = got.reshape(exp.shape)
        # copies are exact; split children within FP32 rounding of the FP64 sample
        np.testing.assert_array_equal(got[~split], exp[~split].astype(np.float32))
        np.testing.assert_allclose(got[split], exp[split], rtol=2e-6, atol=2e-6)


def test_accumulate_matches_oracle():
    import torch
    from paper_2308_04079_amd import _lib
    rules, kw, DC = _rules_pair()
    rng = np.random.default_rng(11)
    n = 3000 + 41
    cams = [scenes.pinhole_camera(w, h) for w, h in ((640, 360), (97, 211), (1920, 1080))]
    V = len(cams)
    tiles = np.where(rng.random((V, n)) < 0.6, rng.integers(1, 9, (V, n)), 0).astype(np.int32)
    i_lo = rng.integers(0, 500, (V, n))
    j_lo = rng.integers(0, 300, (V, n))
    i_hi = i_lo + rng.integers(0, 60, (V, n))
    j_hi = j_lo + rng.integers(0, 60, (V, n))
    rec = np.zeros((V, n, 12), np.float32)
    rec[..., 0] = (i_lo | (j_lo << 16)).astype(np.int32).view(np.float32)
    rec[..., 1] = (i_hi | (j_hi << 16)).astype(np.int32).view(np.float32)
    g2 = rng.normal(0, 1e-4, (V, n, 9)).astype(np.float32)
    # two backward passes into the same statistics
    dc = DC(n)
    dev = torch.device("cuda")
    t_tiles = torch.from_numpy(tiles.ravel()).to(dev)
    t_rec = torch.from_numpy(rec.ravel()).to(dev)
    t_key = torch.zeros(V * n, dtype=torch.int32, device=dev)
    proj = _lib.GsProjected(_lib.ptr(t_key), _lib.ptr(t_tiles), _lib.ptr(t_rec))
    cams_c = _lib.make_cameras(cams)
    t_g2 = torch.from_numpy(g2.ravel()).to(dev)
    dc.accumulate_raw(proj, cams_c, V, n, t_g2)
    dc.accumulate_raw(proj, cams_c, V, n, t_g2)
    torch.cuda.synchronize()
    vis = tiles > 0
    s, c = od.accumulate(g2[..., 0], g2[..., 1], vis, [cm.width for cm in cams],
                         [cm.height for cm in cams])
    np.testing.assert_allclose(to_np(dc.grad_sum), 2 * s, rtol=2e-6, atol=1e-12)
    np.testing.assert_array_equal(to_np(dc.view_count), 2 * c)
    r = np.where(vis, od.screen_radius(i_lo, i_hi, j_lo, j_hi), 0.0).max(0)
    np.testing.assert_array_equal(to_np(dc.max_radius), r)


def test_reset_opacity_and_empty():
    import torch
    from paper_2308_04079_amd import GaussianParams
    from paper_2308_04079_amd.density import DensityControl, reset_opacity
    lg = np.random.default_rng(3).normal(-2, 3, 10000).astype(np.float32)
    t = torch.from_numpy(lg).cuda()
    reset_opacity(t, 0.01)
    np.testing.assert_allclose(to_np(t), od.reset_opacity(lg, 0.01), rtol=1e-6, atol=1e-6)
    # everything removed: an empty model and empty statistics
    sc = scenes.uniform_scene(300, 2, sh_degree=0)
    sc.opacity_logits[:] = -20.0
    dc = DensityControl(300)
    out, src, action = dc.densify(GaussianParams.from_numpy(sc))
    assert out.n == 0 and src.numel() == 0 and int(action.sum()) == 0 and dc.n == 0
