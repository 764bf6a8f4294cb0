"""gs_sort on tile ids written straight into the instance buffers (where the binning's
expansion writes them), for key distributions the rendered scenes reach only by chance:
a single tile, two tiles, a dominant tile, descending ids, block-sized and ragged
counts (including the edges of the per-XCD ranges of key blocks), odd and even numbers
of digit passes, and a count above the capacity. The
result must be the stable sort of the tile ids (values keep their input order within a
tile), with the tile ranges and a longest-first tile order."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2308_04079_amd import _lib

pytestmark = pytest.mark.gpu


def _tiles(kind, n_tiles, m, rng):
    if kind == "random":
        return rng.integers(0, n_tiles, m)
    if kind == "single":
        return np.full(m, n_tiles // 2)
    if kind == "two":
        return rng.choice(np.array([3, n_tiles - 5]), m)
    if kind == "dominant":
        t = np.full(m, n_tiles - 1)
        few = rng.random(m) < 0.1
        t[few] = rng.integers(0, n_tiles, few.sum())
        return t
    if kind == "descending":
        return np.sort(rng.integers(0, n_tiles, m))[::-1].copy()
    raise ValueError(kind)


def _sort(tiles, n_tiles, capacity, count, digit_bits):
    lib = _lib.lib()
    cfg = _lib.default_config(sort_digit_bits=digit_bits)
    passes = -(-int(lib.gs_sort_key_bits(n_tiles)) // digit_bits)
    cap = max(capacity, 1)
    keys = torch.zeros(cap, dtype=torch.int64, device="cuda")
    keys_alt = torch.zeros(cap, dtype=torch.int64, device="cuda")
    vals = torch.zeros(cap, dtype=torch.int32, device="cuda")
    vals_alt = torch.zeros(cap, dtype=torch.int32, device="cuda")
    m_in = min(count, capacity)
    # the expansion's layout: tile ids in the first `capacity` words of keys_alt, values
    # in the buffer from which an even number of passes ends in vals
    keys_alt.view(torch.int32)[:m_in] = torch.as_tensor(tiles[:m_in], dtype=torch.int32)
    src_vals = vals_alt if passes % 2 else vals
    src_vals[:m_in] = torch.arange(m_in, dtype=torch.int32)
    cnt = torch.tensor([count], dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    inst = _lib.GsInstances(_lib.ptr(keys), _lib.ptr(vals), _lib.ptr(keys_alt), _lib.ptr(vals_alt),
                            capacity, _lib.ptr(cnt), _lib.ptr(status))
    ranges = torch.empty(2 * n_tiles, dtype=torch.int32, device="cuda")
    order = torch.empty(n_tiles, dtype=torch.int32, device="cuda")
    ws_bytes = lib.gs_sort_workspace_bytes(capacity, n_tiles, ctypes.byref(cfg))
    ws = torch.empty(max(1, ws_bytes), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    _lib.check("gs_sort", lib.gs_sort(ctypes.byref(inst), n_tiles, ctypes.byref(cfg), _lib.ptr(ranges),
                                      _lib.ptr(order), _lib.ptr(ws), ws.numel(), stream))
    torch.cuda.synchronize()
    addr = lib.gs_sorted_tile_ids(ctypes.byref(inst), n_tiles, ctypes.byref(cfg))
    sorted_ids = None
    for buf in (keys, keys_alt):
        off = (addr - buf.data_ptr()) // 4
        if 0 <= off < 2 * cap:
            sorted_ids = buf.view(torch.int32)[off:off + m_in].cpu().numpy()
    assert sorted_ids is not None
    assert int(status.item()) == 0
    return (sorted_ids.astype(np.int64), vals[:m_in].cpu().numpy().astype(np.int64),
            ranges.cpu().numpy().reshape(-1, 2).astype(np.int64), order.cpu().numpy())


@pytest.mark.parametrize("kind,n_tiles,m,digit_bits", [
    ("random", 32640, 9_000, 8),
    ("random", 32640, 3 * 4096 + 17, 6),      # 15 bits in 3 passes: odd pass count
    ("single", 8160, 50_000, 8),              # every key in one bucket of every pass
    ("two", 8160, 50_000, 7),
    ("dominant", 32640, 60_000, 8),           # one tile holds ~90% of the keys
    ("descending", 8160, 20_000, 8),
    ("random", 300, 4096, 5),                 # exactly one block
    ("random", 300, 4097, 8),                 # one key into a second block
    ("random", 300, 1, 8),
    ("random", 64, 0, 8),
    # the XCD-ordered block mapping: 8 blocks of 3072 keys (one per XCD), one key more
    # (9 blocks: ranges of 2 and 1), and a count whose last XCD range is partial
    ("random", 32640, 8 * 3072, 8),
    ("random", 32640, 8 * 3072 + 1, 8),
    ("dominant", 32640, 1_000_003, 7),
])
def test_stable_tile_sort(kind, n_tiles, m, digit_bits):
    rng = np.random.default_rng(1000 + m + n_tiles)
    tiles = _tiles(kind, n_tiles, m, rng)
    print(f"case {kind} tiles={n_tiles} m={m} bits={digit_bits}", flush=True)
    ids, vals, ranges, order = _sort(tiles, n_tiles, capacity=m + 1000, count=m,
                                     digit_bits=digit_bits)
    perm = np.argsort(tiles, kind="stable")
    assert np.array_equal(ids, tiles[perm])
    assert np.array_equal(vals, perm)
    t = np.arange(n_tiles)
    assert np.array_equal(ranges[:, 0], np.searchsorted(tiles[perm], t))
    assert np.array_equal(ranges[:, 1], np.searchsorted(tiles[perm], t, side="right"))
    assert np.array_equal(np.sort(order), t)
    lens = ranges[order, 1] - ranges[order, 0]
    bucket = np.where(lens > 0, np.floor(np.log2(np.maximum(lens, 1))).astype(int) + 1, 0)
    assert np.all(np.diff(bucket) <= 0)           # longest-list bucket first


def test_count_above_capacity_sorts_the_first_capacity_keys():
    rng = np.random.default_rng(7)
    tiles = rng.integers(0, 8160, 12_000)
    cap = 10_000
    ids, vals, _, _ = _sort(tiles, 8160, capacity=cap, count=12_000, digit_bits=8)
    perm = np.argsort(tiles[:cap], kind="stable")
    assert np.array_equal(ids, tiles[:cap][perm])
    assert np.array_equal(vals, perm)
