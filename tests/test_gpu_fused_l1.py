"""gs_render_bwd_l1 (the L1 loss taken inside the backward blend) against gs_loss_l1
followed by gs_render_bwd on the same forward state, through the C ABI: the screen-space
gradients agree up to the order of the atomic additions (which differs from run to run
in either path), the per-view losses up to the summation order, and the fused loss is
the same bits on every run. Scenes include views of ragged sizes (blocks past the image
edge) and a sparse scene whose waves mostly blend nothing (their pixels still count in
the loss)."""
import numpy as np
import pytest
import torch

import scenes
from paper_2308_04079_amd import GaussianParams, Rasterizer
from paper_2308_04079_amd.raster import l1_loss_grad

pytestmark = pytest.mark.gpu


def _case(n, res, seed, tile):
    sc = scenes.uniform_scene(n, seed, 2, (2.0, 9.0))
    cams = [scenes.pinhole_camera(w, h) for (w, h) in res]
    params = GaussianParams.from_numpy(sc, "cuda")
    tgt = scenes.jitter_means(sc, seed)
    rast = Rasterizer(sh_degree=2, tile_size=tile)
    target = rast.render(GaussianParams.from_numpy(tgt, "cuda"), cams).image.clone()
    return rast, params, cams, target


@pytest.mark.parametrize("n,res,seed,tile", [
    (4000, [(256, 192)], 3, 16),
    (6000, [(320, 200), (131, 97), (64, 64)], 5, 16),
    (5000, [(200, 150), (96, 70)], 7, 8),
    (3000, [(150, 110)], 9, 32),
    (40, [(300, 220), (77, 51)], 11, 16),          # sparse: most waves blend nothing
])
def test_fused_l1_backward_matches_loss_then_backward(n, res, seed, tile):
    rast, params, cams, target = _case(n, res, seed, tile)
    V = len(cams)
    st = rast.render(params, cams)
    print(f"case n={n} views={V} tile={tile}: {int(st.count.item())} instances", flush=True)
    ref_loss = torch.zeros(V, device="cuda")
    dL = l1_loss_grad(st, target, ref_loss)
    ref_grads, ref_g2d = rast.backward(params, st, dL)
    loss = torch.zeros(V, device="cuda")
    grads, g2d = rast.backward(params, st, l1=(target, loss))
    torch.cuda.synchronize()
    a, b = g2d.cpu().numpy(), ref_g2d.cpu().numpy()
    scale = np.abs(b).max() + 1e-30
    assert np.abs(a - b).max() <= 1e-5 * scale
    for k in grads:
        x, y = grads[k].cpu().numpy(), ref_grads[k].cpu().numpy()
        assert np.abs(x - y).max() <= 1e-4 * (np.abs(y).max() + 1e-30), k
    np.testing.assert_allclose(loss.cpu().numpy(), ref_loss.cpu().numpy(), rtol=1e-5, atol=1e-9)

    # the loss is summed in a fixed order: the same bits again; and it is ADDED to the
    # buffer with one float add per view
    again = torch.zeros(V, device="cuda")
    acc = torch.full((V,), 0.25, device="cuda")
    rast.backward(params, st, l1=(target, again))
    rast.backward(params, st, l1=(target, acc))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(again.cpu().numpy(), loss.cpu().numpy())
    np.testing.assert_array_equal(acc.cpu().numpy(), np.float32(0.25) + loss.cpu().numpy())


def test_fused_l1_backward_without_loss_buffer():
    rast, params, cams, target = _case(3000, [(160, 120)], 13, 16)
    st = rast.render(params, cams)
    dL = l1_loss_grad(st, target, None)
    _, ref_g2d = rast.backward(params, st, dL)
    _, g2d = rast.backward(params, st, l1=(target, None))     # no workspace needed
    a, b = g2d.cpu().numpy(), ref_g2d.cpu().numpy()
    assert np.abs(a - b).max() <= 1e-5 * (np.abs(b).max() + 1e-30)
