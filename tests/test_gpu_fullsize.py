"""Parity at the full benchmark size: 3M Gaussians, SH degree 3, 1920x1080, clustered scene.

The launch configuration is the one bench.py times (16x16 tiles, 8-bit sort
digits). Sorted instances and tile ranges are checked bit-exact in full; the
image on a seeded sample of tiles; gradients with dL/dimage restricted to those
tiles (the oracle computes exactly that partial gradient).
"""
import numpy as np
import pytest

import scenes
from oracle.adjoint import render_backward
from oracle.gaussians import project
from oracle.raster import render_tiles, tile_lists
from tests.gpu_common import GROUPS, check_grads, check_view_image, gpu_images, gpu_render, to_np
from tests.test_gpu_parity import check_ranges, check_tile_order, expected_sorted_instances

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    import torch
    sc, cams = scenes.workload("full1080")
    rast, params, state = gpu_render(sc, cams)
    p = project(sc, cams[0])
    tl = tile_lists(p)
    yield sc, cams, rast, params, state, p, tl
    del state, params
    torch.cuda.empty_cache()


def test_full_sort_bit_exact(full):
    sc, cams, rast, params, state, p, tl = full
    M = int(to_np(state.count)[0])
    ek, ev = expected_sorted_instances(state)
    assert M == ek.size
    assert np.array_equal(to_np(state.tile_ids(rast.cfg))[:M].astype(np.int64),
                          (ek >> np.uint64(32)).astype(np.int64))
    assert np.array_equal(to_np(state.vals)[:M].astype(np.int64) & 0xFFFFFFFF, ev)
    check_ranges(state, ek)
    check_tile_order(state)            # 8160 tiles: eight blocks of the order kernels
    # depth keys of every visible Gaussian are the oracle's, bit for bit
    g_valid = to_np(state.tiles_touched)[:sc.n] > 0
    ok = g_valid & p.valid
    assert np.array_equal(to_np(state.depth_key)[:sc.n].view(np.uint32)[ok], p.zkey[ok])
    assert np.array_equal((g_valid ^ p.valid) & ~p.aabb_margin, np.zeros(sc.n, bool))


def sample_tiles(tl, k, seed):
    lens = np.diff(tl.start)
    rng = np.random.default_rng(seed)
    nonempty = np.nonzero(lens > 0)[0]
    picks = set(rng.choice(nonempty, k - 2, replace=False).tolist())
    picks.add(int(np.argmax(lens)))                      # the deepest list
    picks.add(int(tl.tiles_x * tl.tiles_y - 1))          # the ragged bottom-right tile
    return np.array(sorted(picks))


def test_full_image_on_sampled_tiles(full):
    sc, cams, rast, params, state, p, tl = full
    tiles = sample_tiles(tl, 40, 1)
    ref = render_tiles(p, tiles=tiles, tl=tl)
    print(check_view_image(gpu_images(state)[0], p, ref, tl))


def test_full_gradients_on_sampled_tiles(full):
    import torch
    sc, cams, rast, params, state, p, tl = full
    tiles = sample_tiles(tl, 24, 2)
    cam = cams[0]
    ref = render_tiles(p, tiles=tiles, tl=tl)
    w = np.random.default_rng(3).standard_normal((cam.height, cam.width, 3))
    w *= (ref.done & ~ref.ambiguous_grad)[..., None]
    dimg = torch.from_numpy(np.ascontiguousarray(w.transpose(2, 0, 1)).astype(np.float32))
    grads, _ = rast.backward(params, state, dimg.reshape(-1).cuda())
    torch.cuda.synchronize()
    gref, _, _ = render_backward(sc, cam, w, tiles=tiles)
    check_grads({k: to_np(grads[k]) for k in GROUPS}, gref)
