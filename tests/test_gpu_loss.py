"""Photometric loss (Sec. 5.1) on the GPU against the FP64 oracle."""
import numpy as np
import pytest

import scenes
from oracle import loss as ol
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu


def _images(sizes, seed):
    """Smooth seeded images in [0, 1] (render-like) and a perturbed target per view."""
    from scipy import ndimage
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for w, h in sizes:
        x = np.clip(ndimage.gaussian_filter(rng.random((3, h, w)), (0, 2, 2)) * 3 - 1, 0, 1)
        y = np.clip(x + rng.normal(0, 0.05, x.shape), 0, 1)
        y[:, : h // 3] = rng.random((3, h // 3, w))      # a band of unrelated content
        xs.append(x.astype(np.float32))
        ys.append(y.astype(np.float32))
    return xs, ys


def _run(sizes, lam, seed=0):
    import torch
    from paper_2308_04079_amd import _lib
    xs, ys = _images(sizes, seed)
    cams = [scenes.pinhole_camera(w, h) for w, h in sizes]
    cc = _lib.make_cameras(cams)
    x = torch.from_numpy(np.concatenate([a.ravel() for a in xs])).cuda()
    y = torch.from_numpy(np.concatenate([a.ravel() for a in ys])).cuda()
    dL = torch.full_like(x, np.nan)
    loss = torch.zeros(len(sizes), device="cuda")
    lib = _lib.lib()
    ws = torch.empty(lib.gs_loss_workspace_bytes(cc, len(sizes)), dtype=torch.uint8, device="cuda")
    _lib.check("gs_loss_photometric", lib.gs_loss_photometric(
        _lib.ptr(x), _lib.ptr(y), cc, len(sizes), lam, _lib.ptr(dL), _lib.ptr(loss), _lib.ptr(ws),
        ws.numel(), torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return xs, ys, to_np(dL), to_np(loss)


@pytest.mark.parametrize("lam", [0.2, 1.0, 0.0])
def test_photometric_loss_and_gradient_match_oracle(lam):
    # several 32x32 tiles with ragged edges, a view smaller than the window, one tall view
    sizes = [(97, 70), (64, 48), (7, 3), (33, 130)]
    xs, ys, dL, loss = _run(sizes, lam)
    off = 0
    for v, (x, y) in enumerate(zip(xs, ys)):
        L, G = ol.photometric(x.astype(np.float64), y.astype(np.float64), lam)
        g = dL[off:off + x.size].reshape(x.shape)
        off += x.size
        assert abs(loss[v] - L) <= 2e-6 * max(1.0, abs(L)), (v, loss[v], L)
        assert rel_l2(g, G) <= 1e-4, (v, rel_l2(g, G))
        assert np.abs(g - G).max() <= 1e-3 * np.abs(G).max() + 1e-12
    assert off == dL.size


def test_photometric_loss_at_1080p():
    xs, ys, dL, loss = _run([(1920, 1080)], 0.2, seed=3)
    L, G = ol.photometric(xs[0].astype(np.float64), ys[0].astype(np.float64), 0.2)
    assert abs(loss[0] - L) <= 1e-5 * abs(L)
    assert rel_l2(dL.reshape(G.shape), G) <= 1e-4


def test_identical_images_give_zero_loss():
    import torch
    from paper_2308_04079_amd import _lib
    sizes = [(50, 40)]
    xs, _ = _images(sizes, 5)
    cc = _lib.make_cameras([scenes.pinhole_camera(50, 40)])
    x = torch.from_numpy(xs[0].ravel()).cuda()
    dL = torch.empty_like(x)
    loss = torch.zeros(1, device="cuda")
    lib = _lib.lib()
    ws = torch.empty(lib.gs_loss_workspace_bytes(cc, 1), dtype=torch.uint8, device="cuda")
    assert lib.gs_loss_photometric(_lib.ptr(x), _lib.ptr(x), cc, 1, 0.2, _lib.ptr(dL),
                                   _lib.ptr(loss), _lib.ptr(ws), ws.numel(), None) == 0
    torch.cuda.synchronize()
    assert abs(float(loss[0])) < 1e-6
    assert float(dL.abs().max()) < 1e-7
