"""Autotuner for the knobs that change speed but not results.

Tile size (8, 16, 32; the image is tile-size independent because a Gaussian reaches a
pixel only inside its 3-sigma ellipse), the LDS batch depth of the blend kernels (32, 64
or 128 list entries staged per wave and round) and the radix digit width of the sort (6, 7,
8 bits; the sort is stable either way) are timed on the caller's own scene and views,
one full step (forward, L1 gradient, backward) per trial, and the fastest combination
is kept in a JSON cache keyed by device, Gaussian count (power-of-two bucket), SH
degree and the view resolutions.
"""
from __future__ import annotations

import json
import math
import os

import torch

from .raster import Rasterizer

TILE_SIZES = (8, 16, 32)
LDS_BATCHES = (32, 64, 128)
DIGIT_BITS = (6, 7, 8)


def cache_path() -> str:
    return os.environ.get("GS_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gs_mi355x",
                                       "autotune.json"))


def cache_key(params, cams) -> str:
    dev = torch.cuda.get_device_name(params.means.device)
    nb = int(math.log2(max(params.n, 1)))
    res = ",".join(sorted(f"{c.width}x{c.height}" for c in cams))
    return f"{dev}|n2^{nb}|sh{params.sh_degree}|{res}"


def time_step(rast: Rasterizer, params, cams, target, steps: int) -> float:
    """Milliseconds of one forward + backward with the L1 loss, averaged over ``steps``."""
    state = rast.render(params, cams)                     # sizes the capacity
    rast.capacity = int(state.read_status()[1] * 1.15) + 4096
    loss = torch.zeros(len(cams), device=params.means.device)

    def one():
        st = rast.render(params, cams, check=False)
        rast.backward(params, st, l1=(target, loss))
    one()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        one()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def autotune(params, cams, target=None, steps: int = 3, use_cache: bool = True,
             tile_sizes=TILE_SIZES, lds_batches=LDS_BATCHES, digit_bits=DIGIT_BITS,
             bg=(0.0, 0.0, 0.0)) -> dict:
    """Best {"tile_size", "lds_batch", "sort_digit_bits", "ms"} for these params and views."""
    key = cache_key(params, cams)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    if target is None:
        target = torch.zeros(3 * sum(c.width * c.height for c in cams), device=params.means.device)
    trials = []
    for ts in tile_sizes:
        for lb in lds_batches:
            for db in digit_bits:
                rast = Rasterizer(sh_degree=params.sh_degree, tile_size=ts, bg=bg,
                                  sort_digit_bits=db, lds_batch=lb)
                trials.append({"tile_size": ts, "lds_batch": lb, "sort_digit_bits": db,
                               "ms": time_step(rast, params, cams, target, steps)})
    best = min(trials, key=lambda t: t["ms"])
    best = dict(best, trials=trials)
    if use_cache:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        cache[key] = best
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return best


def tuned_rasterizer(params, cams, target=None, **kw) -> Rasterizer:
    best = autotune(params, cams, target, **kw)
    return Rasterizer(sh_degree=params.sh_degree, tile_size=best["tile_size"],
                      sort_digit_bits=best["sort_digit_bits"], lds_batch=best["lds_batch"],
                      bg=kw.get("bg", (0.0, 0.0, 0.0)))
