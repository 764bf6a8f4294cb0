"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Bars: depth keys, pixel boxes, tile lists, sorted instances and tile ranges
bit-exact (decisions within the oracle's margins excepted); images within 1e-4
max-abs, T_final within its rounding bound and the same last contributor, where a
pixel with a decision within its margin must equal one of its legitimate outcomes;
gradients within 1e-3 relative L2 per group and element-wise within 1e-3 of the
group's largest magnitude.
"""
import math

import numpy as np
import pytest

import scenes
from oracle.adjoint import render_backward
from oracle.gaussians import project
from oracle.raster import render_tiles, tile_lists
from oracle.rules import Rules
from tests.gpu_common import (GROUPS, TOL_GRAD, TOL_IMAGE, check_grads, check_view_image,
                              decode_records, gpu_images, gpu_render, rel_l2, to_np)

pytestmark = pytest.mark.gpu


def small_cases():
    return {
        "small": scenes.workload("small"),
        "ragged": (scenes.uniform_scene(700, 21, 2, (2.0, 8.0)), [scenes.pinhole_camera(77, 45)]),
        "offcentre": (scenes.uniform_scene(900, 22, 3, (1.5, 9.0), xy_range=(-2, 2)),
                      [scenes.look_at_camera([0.4, -0.3, -0.5], [0.0, 0.1, 5.0], 96, 64)]),
    }


CASES = small_cases()


@pytest.mark.parametrize("name", list(CASES))
def test_project_matches_oracle(name):
    sc, cams = CASES[name]
    _, _, state = gpu_render(sc, cams)
    p = project(sc, cams[0])
    g = decode_records(state, 0)
    flagged = p.aabb_margin
    assert np.array_equal(g["valid"] & ~flagged, p.valid & ~flagged)
    ok = g["valid"] & p.valid
    assert np.array_equal(g["zkey"][ok], p.zkey[ok])
    for k in ("i_lo", "i_hi", "j_lo", "j_hi"):
        assert np.array_equal(g[k][ok & ~flagged], getattr(p, k)[ok & ~flagged]), k
    np.testing.assert_allclose(g["u"][ok], p.u[ok], rtol=0, atol=2e-5)
    np.testing.assert_allclose(g["v"][ok], p.v[ok], rtol=0, atol=2e-5)
    np.testing.assert_allclose(g["conic"][ok], p.conic[ok], rtol=2e-5,
                               atol=2e-6 * np.abs(p.conic[ok]).max())
    np.testing.assert_allclose(g["opacity"][ok], p.opacity[ok], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(g["rgb"][ok], p.rgb[ok], rtol=0, atol=1e-6)


def expected_sorted_instances(state, tile=16):
    """Instances built in NumPy from the GPU's own projection, sorted by the paper's
    single key (tile << 32 | depth), ties by value."""
    keys, vals = [], []
    for v, cam in enumerate(state.cams):
        g = decode_records(state, v)
        tx_n = (cam.width + tile - 1) // tile
        ids = np.nonzero(g["valid"])[0]
        tx0, tx1 = g["i_lo"][ids] // tile, g["i_hi"][ids] // tile
        ty0, ty1 = g["j_lo"][ids] // tile, g["j_hi"][ids] // tile
        w = tx1 - tx0 + 1
        cnt = w * (ty1 - ty0 + 1)
        own = np.repeat(np.arange(ids.size), cnt)
        local = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        t = state.tile_offset[v] + (ty0[own] + local // w[own]) * tx_n + tx0[own] + local % w[own]
        keys.append((t.astype(np.uint64) << np.uint64(32)) | g["zkey"][ids][own].astype(np.uint64))
        vals.append(v * state.n + ids[own])
    keys = np.concatenate(keys) if keys else np.zeros(0, np.uint64)
    vals = np.concatenate(vals).astype(np.int64) if vals else np.zeros(0, np.int64)
    order = np.lexsort((vals, keys))
    return keys[order], vals[order]


@pytest.mark.parametrize("name", list(CASES))
def test_sort_and_ranges_bit_exact(name):
    sc, cams = CASES[name]
    rast, _, state = gpu_render(sc, cams)
    M = int(to_np(state.count)[0])
    ek, ev = expected_sorted_instances(state)
    assert M == ek.size
    gt = to_np(state.tile_ids(rast.cfg))[:M].astype(np.int64)
    gv = to_np(state.vals)[:M].astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(gt, (ek >> np.uint64(32)).astype(np.int64))
    assert np.array_equal(gv, ev)
    check_ranges(state, ek)


def check_ranges(state, ek):
    rng = to_np(state.ranges).reshape(-1, 2).astype(np.int64)
    tiles = (ek >> np.uint64(32)).astype(np.int64)
    t = np.arange(state.n_tiles)
    assert np.array_equal(rng[:, 0], np.searchsorted(tiles, t))
    assert np.array_equal(rng[:, 1], np.searchsorted(tiles, t, side="right"))


@pytest.mark.parametrize("name", list(CASES))
def test_tile_lists_match_oracle(name):
    sc, cams = CASES[name]
    _, _, state = gpu_render(sc, cams)
    p = project(sc, cams[0])
    tl = tile_lists(p)
    rng = to_np(state.ranges).reshape(-1, 2).astype(np.int64)
    vals = to_np(state.vals).astype(np.int64) & 0xFFFFFFFF
    for t in range(tl.tiles_x * tl.tiles_y):
        gids = vals[rng[t, 0]:rng[t, 1]]
        oids = tl.ids[tl.start[t]:tl.start[t + 1]]
        keep_g = gids[~p.aabb_margin[gids]]
        keep_o = oids[~p.aabb_margin[oids]]
        assert np.array_equal(keep_g, keep_o), t


def compare_images(state, sc, cams, tiles=None, rules=Rules()):
    worst = 0.0
    for v, gpu in enumerate(gpu_images(state)):
        p = project(sc, cams[v], rules)
        tl = tile_lists(p, rules)
        ref = render_tiles(p, rules, tiles=tiles, tl=tl)
        worst = max(worst, check_view_image(gpu, p, ref, tl, rules)["worst"])
    return worst


@pytest.mark.parametrize("name", list(CASES))
def test_forward_image_matches_oracle(name):
    sc, cams = CASES[name]
    _, _, state = gpu_render(sc, cams)
    compare_images(state, sc, cams)


@pytest.mark.parametrize("tile,batch", [(8, 64), (32, 64), (16, 128), (8, 128), (16, 32),
                                        (32, 32)])
def test_tile_size_and_batch_depth_do_not_change_image(tile, batch):
    sc, cams = CASES["ragged"]
    _, _, s16 = gpu_render(sc, cams)
    _, _, st = gpu_render(sc, cams, tile_size=tile, lds_batch=batch)
    a, b = gpu_images(s16)[0], gpu_images(st)[0]
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    compare_images(st, sc, cams, rules=Rules(tile=tile))


def backward_case(sc, cams, seed, tiles=None, **cfg):
    import torch
    rast, params, state = gpu_render(sc, cams, **cfg)
    cam = cams[0]
    ref = render_tiles(project(sc, cam), tiles=tiles)
    w = np.random.default_rng(seed).standard_normal((cam.height, cam.width, 3))
    w *= (ref.done & ~ref.ambiguous_grad)[..., None]
    dimg = torch.from_numpy(np.ascontiguousarray(w.transpose(2, 0, 1)).astype(np.float32))
    grads, grad2d = rast.backward(params, state, dimg.reshape(-1).cuda())
    torch.cuda.synchronize()
    gref, acc, p = render_backward(sc, cam, w, tiles=tiles)
    return grads, grad2d, gref, acc, p


@pytest.mark.parametrize("name,cfg", [(n, {}) for n in CASES] +
                         [("offcentre", {"lds_batch": 128}), ("ragged", {"tile_size": 32}),
                          ("small", {"tile_size": 8}),
                          ("offcentre", {"tile_size": 8, "lds_batch": 128}),
                          ("ragged", {"tile_size": 32, "lds_batch": 128}),
                          ("ragged", {"lds_batch": 32}), ("offcentre", {"tile_size": 8, "lds_batch": 32})])
def test_backward_matches_oracle(name, cfg):
    sc, cams = CASES[name]
    grads, grad2d, gref, acc, p = backward_case(sc, cams, 5, **cfg)
    g2 = to_np(grad2d).reshape(-1, 9)[:sc.n].astype(np.float64)
    ok = p.valid
    check_grads({"u": g2[ok, 0], "v": g2[ok, 1], "opacity": g2[ok, 5], "rgb": g2[ok, 6:9]},
                {"u": acc["u"][ok], "v": acc["v"][ok], "opacity": acc["opacity"][ok],
                 "rgb": acc["rgb"][ok]}, ("u", "v", "opacity", "rgb"))
    check_grads({k: to_np(grads[k]) for k in GROUPS}, gref)


def test_single720_sampled_tiles_forward_and_backward():
    sc, cams = scenes.workload("single720")
    rng = np.random.default_rng(7)
    tl_x, tl_y = 80, 45
    tiles = np.sort(rng.choice(tl_x * tl_y, 120, replace=False))
    _, _, state = gpu_render(sc, cams)
    compare_images(state, sc, cams, tiles=tiles)
    grads, _, gref, _, _ = backward_case(sc, cams, 6, tiles=tiles)
    check_grads({k: to_np(grads[k]) for k in GROUPS}, gref)


def test_multiview_batch_equals_single_views():
    sc = scenes.clustered_scene(20_000, 31, 3)
    cams = scenes.orbit_cameras(3, 31, resolutions=((96, 64), (64, 48), (128, 72)))
    _, _, batch = gpu_render(sc, cams)
    check_tile_order(batch)
    bimgs = gpu_images(batch)
    for v, cam in enumerate(cams):
        _, _, single = gpu_render(sc, [cam])
        s = gpu_images(single)[0]
        np.testing.assert_array_equal(bimgs[v][0], s[0])
        np.testing.assert_array_equal(bimgs[v][1], s[1])
        np.testing.assert_array_equal(bimgs[v][2], s[2])
    compare_images(batch, sc, cams)


def test_empty_and_fully_culled_scenes():
    cam = scenes.pinhole_camera(40, 24)
    empty = scenes.uniform_scene(0, 1, 0)
    _, _, st = gpu_render(empty, [cam])
    img, T, gid = gpu_images(st)[0]
    assert np.all(img == 0) and np.all(T == 1) and np.all(gid == -1)
    behind = scenes.uniform_scene(200, 2, 0, (-5.0, -1.0))
    _, _, st = gpu_render(behind, [cam])
    img, T, gid = gpu_images(st)[0]
    assert int(to_np(st.count)[0]) == 0 and np.all(img == 0) and np.all(gid == -1)


def test_capacity_overflow_is_reported_and_recovered():
    from paper_2308_04079_amd import GaussianParams, Rasterizer
    sc, cams = CASES["small"]
    params = GaussianParams.from_numpy(sc, "cuda")
    rast = Rasterizer(sh_degree=0, capacity=16)
    state = rast.render(params, cams, check=False)
    st, ct = state.read_status()
    assert st & 1 and ct > 16
    state = rast.render(params, cams)        # grows the capacity and re-runs
    assert rast.capacity >= ct
    compare_images(state, sc, cams)


def expected_clamped_instances(state, cap, tile=16):
    """What gs_bin + gs_sort produce when the capacity is short: the first `cap` visible
    pairs in index order, sorted by (depth, index), expanded row-major into their
    tiles, the first `cap` instances kept, then sorted stably by tile id."""
    recs = [decode_records(state, v) for v in range(state.n_views)]
    ids = [np.nonzero(g["valid"])[0] for g in recs]
    view = np.concatenate([np.full(i.size, v) for v, i in enumerate(ids)])
    local = np.concatenate(ids)
    zkey = np.concatenate([g["zkey"][i] for g, i in zip(recs, ids)])
    gidx = view * state.n + local
    keep = min(gidx.size, cap)
    view, local, zkey, gidx = view[:keep], local[:keep], zkey[:keep], gidx[:keep]
    tiles, vals = [], []
    for k in np.lexsort((gidx, zkey)):
        g, i = recs[view[k]], local[k]
        tx_n = (state.cams[view[k]].width + tile - 1) // tile
        for ty in range(g["j_lo"][i] // tile, g["j_hi"][i] // tile + 1):
            for tx in range(g["i_lo"][i] // tile, g["i_hi"][i] // tile + 1):
                tiles.append(state.tile_offset[view[k]] + ty * tx_n + tx)
                vals.append(gidx[k])
        if len(tiles) >= cap:
            break
    tiles, vals = np.array(tiles[:cap], np.int64), np.array(vals[:cap], np.int64)
    perm = np.argsort(tiles, kind="stable")
    return tiles[perm], vals[perm]


@pytest.mark.parametrize("short", [0.3, 0.97])
def test_a_short_capacity_over_several_expansion_blocks(short):
    """Capacity below the instance count (25k) by several 2048-instance expansion blocks
    (at 0.3 below the 12k visible pairs as well): the status bit, the exact count, and
    the instances written are the clamped expansion, sorted by tile."""
    from paper_2308_04079_amd import GaussianParams, Rasterizer
    sc = scenes.uniform_scene(6000, 62, 1, (2.0, 6.0))
    cams = [scenes.pinhole_camera(160, 120), scenes.pinhole_camera(96, 64)]
    params = GaussianParams.from_numpy(sc, "cuda")
    full = Rasterizer(sh_degree=1).render(params, cams)
    st, ct = full.read_status()
    assert st == 0 and ct > 4 * 2048
    cap = int(ct * short)
    rast = Rasterizer(sh_degree=1, capacity=cap)
    state = rast.render(params, cams, check=False)
    st2, ct2 = state.read_status()
    assert st2 & 1 and ct2 == ct
    et, ev = expected_clamped_instances(state, cap)
    assert et.size == cap
    assert np.array_equal(to_np(state.tile_ids(rast.cfg))[:cap].astype(np.int64), et)
    assert np.array_equal(to_np(state.vals)[:cap].astype(np.int64) & 0xFFFFFFFF, ev)


def test_degenerate_gaussians_do_not_poison_the_image():
    sc = scenes.uniform_scene(300, 41, 1, (2.0, 6.0))
    sc.quats[:, :10] = 0.0                    # zero quaternion: culled
    sc.means[0, 10:20] = np.nan               # non-finite: culled
    sc.log_scales[:, 20:30] = -30.0           # vanishing scale: culled (empty box or det)
    sc.opacity_logits[30:35] = -800.0         # sigmoid far below any alpha_min: opacity 0
    sc.opacity_logits[35:40] = 800.0          # sigmoid 1: every alpha at the clamp
    sc.sh[2, 1, 40:45] = np.inf               # a non-finite colour coefficient: culled
    sc.sh[0, 0, 45:48] = np.nan
    cams = [scenes.pinhole_camera(64, 64)]
    _, _, state = gpu_render(sc, cams)
    img = gpu_images(state)[0][0]
    assert np.isfinite(img).all()
    assert np.all(to_np(state.tiles_touched)[:20] == 0)
    assert np.all(to_np(state.tiles_touched)[40:48] == 0)
    g = decode_records(state, 0)
    assert np.all(g["opacity"][30:35][g["valid"][30:35]] == 0.0)
    assert np.all(g["opacity"][35:40][g["valid"][35:40]] == 1.0)
    compare_images(state, sc, cams)


def test_l1_loss_gradient():
    import torch
    from paper_2308_04079_amd.raster import l1_loss_grad
    sc = scenes.uniform_scene(500, 51, 1, (2.0, 6.0))
    cams = [scenes.pinhole_camera(40, 30), scenes.pinhole_camera(23, 17)]
    _, _, state = gpu_render(sc, cams)
    target = torch.rand_like(state.image)
    target[:7] = state.image[:7]                      # exact ties give a zero gradient
    loss = torch.zeros(2, device="cuda")
    dL = to_np(l1_loss_grad(state, target, loss)).astype(np.float64)
    img, tgt = to_np(state.image).astype(np.float64), to_np(target).astype(np.float64)
    for v, cam in enumerate(cams):
        sl = slice(3 * state.pix_offset[v], 3 * state.pix_offset[v + 1])
        k = 3 * cam.width * cam.height
        np.testing.assert_allclose(dL[sl], np.sign(img[sl] - tgt[sl]) / k, rtol=1e-6, atol=0)
        np.testing.assert_allclose(to_np(loss)[v], np.abs(img[sl] - tgt[sl]).mean(), rtol=1e-5)


def test_backward_walk_is_bounded_by_the_tile_list():
    """A last_idx past its tile's instance list acts as the list's last entry: the
    backward walk starts there, and the gradients equal those of that clamped input."""
    import dataclasses

    import torch
    sc, cams = CASES["ragged"]
    rast, params, state = gpu_render(sc, cams)
    cam = cams[0]
    W, H, T = cam.width, cam.height, 16
    ranges = to_np(state.ranges).astype(np.int64).reshape(-1, 2)
    last = to_np(state.last_idx).astype(np.int64)
    ys, xs = np.divmod(np.arange(W * H), W)
    tile = state.tile_offset[0] + (ys // T) * ((W + T - 1) // T) + xs // T
    hit = last >= 0
    assert hit.sum() > 100
    huge = np.where(hit, 2 ** 31 - 1, last)
    clamped = np.where(hit, ranges[tile, 1] - 1, last)
    w = np.random.default_rng(7).standard_normal(3 * W * H).astype(np.float32)
    dimg = torch.from_numpy(w).cuda()
    out = []
    for li in (huge, clamped):
        st = dataclasses.replace(state, last_idx=torch.from_numpy(li.astype(np.int32)).cuda())
        grads, _ = rast.backward(params, st, dimg)
        torch.cuda.synchronize()
        out.append({k: to_np(grads[k]).astype(np.float64) for k in GROUPS})
    for k in GROUPS:
        assert np.abs(out[0][k]).max() > 0, k
        assert rel_l2(out[0][k], out[1][k]) <= 1e-5, k


def test_blend_kernels_clip_ranges_and_tile_order_they_did_not_get_from_the_sort():
    """Tile ranges and a tile order that gs_sort did not write are clipped by the
    kernels: every list becomes [0, capacity) (values past the instance count are
    whatever the buffer holds; entries >= V N are skipped), tile-order entries that are
    no tile id issue nothing. The calls complete and what they write is finite."""
    import ctypes
    import dataclasses

    import torch
    from paper_2308_04079_amd import _lib
    sc, cams = CASES["ragged"]
    rast, params, state = gpu_render(sc, cams)
    ranges = state.ranges.clone().view(-1, 2)
    ranges[:, 0] = 0
    ranges[:, 1] = -1                                   # 0xFFFFFFFF
    order = state.order.clone()
    order[::3] = -1                                     # not a tile id: skipped
    bad = dataclasses.replace(state, ranges=ranges.reshape(-1), order=order)
    image = torch.full_like(state.image, 7.0)
    lib = _lib.lib()
    proj = _lib.GsProjected(_lib.ptr(bad.depth_key), _lib.ptr(bad.tiles_touched),
                            _lib.ptr(bad.record))
    inst = bad.instances()
    stream = torch.cuda.current_stream().cuda_stream
    _lib.check("gs_render_fwd", lib.gs_render_fwd(
        ctypes.byref(proj), ctypes.byref(inst), _lib.ptr(bad.ranges), _lib.ptr(bad.order),
        bad.cams_c, bad.n_views, ctypes.byref(rast.cfg), _lib.ptr(image), _lib.ptr(bad.T_final),
        _lib.ptr(bad.last_idx), bad.n, stream))
    torch.cuda.synchronize()
    img = to_np(image)
    assert np.isfinite(img).all()
    assert (img == 7.0).any() and (img != 7.0).any()   # skipped tiles kept the fill
    last = to_np(bad.last_idx)
    assert last.max() < bad.capacity
    w = torch.ones(state.image.numel(), device="cuda")
    grads, _ = rast.backward(params, bad, w)
    torch.cuda.synchronize()
    for k in GROUPS:
        assert np.isfinite(to_np(grads[k])).all(), k


def check_tile_order(state):
    """The issue order is a permutation of the tile ids, longest-list bucket first."""
    order = to_np(state.order).astype(np.int64)
    r = to_np(state.ranges).astype(np.int64).reshape(-1, 2)
    assert np.array_equal(np.sort(order), np.arange(state.n_tiles))
    lens = r[order, 1] - r[order, 0]
    bucket = np.where(lens > 0, np.floor(np.log2(np.maximum(lens, 1))).astype(np.int64) + 1, 0)
    assert np.all(np.diff(bucket) <= 0)


@pytest.mark.parametrize("name", list(CASES))
def test_tile_order_is_longest_first(name):
    sc, cams = CASES[name]
    _, _, state = gpu_render(sc, cams)
    check_tile_order(state)


def test_the_largest_view_batch_equals_single_views():
    """GS_MAX_VIEWS (32) views of mixed small sizes in one call of every stage give the
    same images, transmittances and last contributors as 32 single-view calls."""
    from paper_2308_04079_amd import _lib
    sc = scenes.clustered_scene(5_000, 33, 1)
    cams = scenes.orbit_cameras(32, 33, resolutions=((40, 24), (17, 33), (64, 16), (8, 8)))
    assert len(cams) == 32 == _lib.MAX_VIEWS
    _, _, batch = gpu_render(sc, cams)
    check_tile_order(batch)
    bimgs = gpu_images(batch)
    for v, cam in enumerate(cams):
        _, _, single = gpu_render(sc, [cam])
        s = gpu_images(single)[0]
        for a, b in zip(bimgs[v], s):
            np.testing.assert_array_equal(a, b)
    compare_images(batch, sc, cams)


def test_a_very_wide_image():
    """A 32000 x 12 view (2000 x 1 tiles at 16 pixels, a ragged bottom row): tile lists,
    image and transmittance against the oracle on sampled tiles."""
    sc = scenes.uniform_scene(4000, 34, 1, (2.0, 8.0))
    sc.means[0] *= 60.0                                   # spread along the image's width
    sc.means[1] *= 0.05                                   # and close to its 12-pixel strip
    cam = scenes.pinhole_camera(32000, 12, fov_y_deg=2.0)
    _, _, state = gpu_render(sc, [cam])
    ek, _ = expected_sorted_instances(state)
    check_ranges(state, ek)
    check_tile_order(state)            # 2000 tiles: a full and a ragged order block
    p = project(sc, cam)
    tl = tile_lists(p)
    lens = np.diff(tl.start)
    nonempty = np.nonzero(lens > 0)[0]
    assert nonempty.size > 20
    tiles = np.unique(np.concatenate([nonempty[:: max(1, nonempty.size // 20)], [tl.tiles_x - 1]]))
    ref = render_tiles(p, tiles=tiles, tl=tl)
    assert ref.done.sum() > 1000
    check_view_image(gpu_images(state)[0], p, ref, tl)


def test_gaussians_larger_than_the_image():
    """A few Gaussians whose 3-sigma boxes cover the whole view (clamped to it: every tile
    lists them) among ordinary ones: sort, image and gradients against the oracle."""
    sc = scenes.uniform_scene(600, 37, 1, (2.0, 6.0))
    sc.log_scales[:, :5] = np.log(3.0)                    # 3 world units at depth 2-6
    sc.opacity_logits[:5] = -3.0                          # faint, so the rest shows through
    cams = [scenes.pinhole_camera(80, 56)]
    _, _, state = gpu_render(sc, cams)
    tt = to_np(state.tiles_touched)
    assert (tt[:5] == 5 * 4).sum() >= 3                   # 80x56 at 16 px: 5 x 4 tiles
    ek, ev = expected_sorted_instances(state)
    M = int(to_np(state.count)[0])
    assert np.array_equal(to_np(state.vals)[:M].astype(np.int64) & 0xFFFFFFFF, ev)
    compare_images(state, sc, cams)
    grads, grad2d, gref, acc, p = backward_case(sc, cams, 8)
    check_grads({k: to_np(grads[k]) for k in GROUPS}, gref)
