"""gs_sort_noalloc (the sort with the library's static scratch) against gs_sort with a
caller workspace, through the C ABI, on the same freshly binned instances: tile ranges,
sorted tile ids and sorted instance values bit for bit, and the tile issue order a
permutation with the same longest-list-first bucket sequence (the order inside a bucket
is arbitrary). Two calls in a row, the second on a smaller input, so that the second
runs on scratch the first one left behind."""
import ctypes

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu


def _sorted_pair(sc, cams, tile_size):
    import torch

    from paper_2308_04079_amd import GaussianParams, Rasterizer, _lib
    lib = _lib.lib()
    params = GaussianParams.from_numpy(sc, "cuda")
    rast = Rasterizer(sh_degree=sc.sh_degree, tile_size=tile_size)
    st = rast.render(params, cams)
    stream = torch.cuda.current_stream().cuda_stream
    cfg = ctypes.byref(rast.cfg)
    proj, inst = st.projected(), st.instances()
    V, n = st.n_views, st.n
    bin_ws = torch.empty(max(1, lib.gs_bin_workspace_bytes(V * n, cfg)), dtype=torch.uint8,
                         device="cuda")
    need = lib.gs_sort_workspace_bytes(st.capacity, st.n_tiles, cfg)
    assert 0 < need <= _lib.SORT_SCRATCH_BYTES
    sort_ws = torch.empty(need, dtype=torch.uint8, device="cuda")

    def rebin():
        st.status.zero_()
        _lib.check("gs_bin", lib.gs_bin(ctypes.byref(proj), n, st.cams_c, V, cfg, ctypes.byref(inst),
                                        _lib.ptr(bin_ws), bin_ws.numel(), stream))

    def outputs():
        torch.cuda.synchronize()
        stat, count = st.read_status()
        assert stat == 0, stat
        ranges = st.ranges.view(-1, 2).cpu().numpy().copy()
        order = st.order.cpu().numpy().copy()
        vals = st.vals[:count].cpu().numpy().copy()
        tiles = st.tile_ids(rast.cfg)[:count].cpu().numpy().copy()
        return ranges, order, vals, tiles

    rebin()
    st.ranges.fill_(0x7FFFFFFF)
    st.order.fill_(0x7FFFFFFF)
    _lib.check("gs_sort", lib.gs_sort(ctypes.byref(inst), st.n_tiles, cfg, _lib.ptr(st.ranges),
                                      _lib.ptr(st.order), _lib.ptr(sort_ws), sort_ws.numel(),
                                      stream))
    ref = outputs()
    rebin()
    st.ranges.fill_(0x7FFFFFFF)
    st.order.fill_(0x7FFFFFFF)
    _lib.check("gs_sort_noalloc", lib.gs_sort_noalloc(ctypes.byref(inst), st.n_tiles, cfg,
                                                      _lib.ptr(st.ranges), _lib.ptr(st.order),
                                                      stream))
    got = outputs()
    return ref, got, st.n_tiles


def _bucket(ranges):
    ln = (ranges[:, 1] - ranges[:, 0]).astype(np.int64)
    return np.where(ln > 0, np.floor(np.log2(np.maximum(ln, 1))).astype(np.int64) + 1, 0)


@pytest.mark.parametrize("first,second", [((20000, 640, 480, 16), (3000, 200, 136, 16)),
                                          ((12000, 512, 384, 8), (2500, 160, 120, 32))])
def test_noalloc_sort_matches_workspace_sort(first, second):
    for n, w, h, tile in (first, second):
        sc = scenes.uniform_scene(n, n % 97, 1, (2.0, 8.0))
        cams = [scenes.pinhole_camera(w, h)]
        (r_ranges, r_order, r_vals, r_tiles), (g_ranges, g_order, g_vals, g_tiles), n_tiles = \
            _sorted_pair(sc, cams, tile)
        print(f"case n={n} {w}x{h} tile {tile}: {r_vals.size} instances, {n_tiles} tiles",
              flush=True)
        assert r_vals.size > 0
        np.testing.assert_array_equal(g_ranges, r_ranges)
        np.testing.assert_array_equal(g_vals, r_vals)
        np.testing.assert_array_equal(g_tiles, r_tiles)
        # issue order: a permutation of the tiles, longest-list bucket first, the same
        # bucket sequence as the workspace sort's
        assert np.array_equal(np.sort(g_order), np.arange(n_tiles))
        b = _bucket(r_ranges)
        np.testing.assert_array_equal(b[g_order], b[r_order])
        assert np.all(np.diff(b[g_order]) <= 0)
