"""Depth keys, tile lists and front-to-back blending in FP64 (oracle side; test infrastructure only).

Follows Sec. 6 and App. C / Alg. 2 (CreateTiles, DuplicateWithKeys, SortByKeys,
IdentifyTileRanges, BlendInOrder) and the image-formation model
C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j) (Eq. front-to-back, read with the
product over j < i). Blending rules are those of App. C ("Numerical stability"):

* alpha_i = min(0.99, o_i exp(-m/2)) with m the Mahalanobis distance of the pixel
  centre; pixels outside the 3-sigma ellipse (m > 9) are not touched (reading);
* a Gaussian whose alpha is below 1/255 is skipped;
* before blending, T' = T (1 - alpha) is formed; if T' < 1e-4 the pixel stops and
  this Gaussian is not blended;
* the background is added as T_final * bg (reading; black unless stated).

Ties in depth are broken by Gaussian index (a stable sort of the instances,
which are created in index order). The per-pixel "last contributor" is recorded
as the list position of the last blended Gaussian.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .rules import Rules


def sort_order(proj, mask=None) -> np.ndarray:
    """Gaussian ids ordered by (depth bits, id): the within-tile order of Alg. 2."""
    mask = proj.valid if mask is None else mask
    ids = np.nonzero(mask)[0]
    order = np.lexsort((ids, proj.zkey[ids].astype(np.int64)))
    return ids[order]


@dataclasses.dataclass
class TileLists:
    tiles_x: int
    tiles_y: int
    start: np.ndarray   # (n_tiles + 1,) CSR offsets
    ids: np.ndarray     # Gaussian ids, tile-major, depth order inside each tile
    flagged: np.ndarray  # per entry: membership depends on an AABB bound within margin


def tile_lists(proj, rules: Rules = Rules()) -> TileLists:
    """Per tile, the ids of the Gaussians whose pixel AABB covers a pixel of the tile.

    The instance key is (tile id, depth bits) with the tile id in the high bits
    (App. C, "Sorting"); sorting all instances by it is the same as listing, per
    tile, the Gaussians of that tile in global depth order.
    """
    T = rules.tile
    tiles_x = (proj.width + T - 1) // T
    tiles_y = (proj.height + T - 1) // T
    order = sort_order(proj)
    tx0, tx1 = proj.tx0[order], proj.tx1[order]
    ty0, ty1 = proj.ty0[order], proj.ty1[order]
    cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1)
    total = int(cnt.sum())
    owner = np.repeat(np.arange(order.size), cnt)
    first = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(total) - first
    w = (tx1 - tx0 + 1)[owner]
    tx = tx0[owner] + local % w
    ty = ty0[owner] + local // w
    tile = ty * tiles_x + tx
    # stable by tile: keeps the depth order of `order` inside each tile
    perm = np.argsort(tile, kind="stable")
    tile_sorted = tile[perm]
    ids = order[owner[perm]]
    start = np.searchsorted(tile_sorted, np.arange(tiles_x * tiles_y + 1))
    flagged = proj.aabb_margin[ids]
    return TileLists(tiles_x, tiles_y, start, ids, flagged)


@dataclasses.dataclass
class BlendResult:
    color: np.ndarray      # (P, 3)
    T_final: np.ndarray    # (P,)
    last_pos: np.ndarray   # (P,) list position of the last blended Gaussian, -1 if none
    last_id: np.ndarray    # (P,) Gaussian id of the last blended Gaussian, -1 if none
    n_eval: np.ndarray     # (P,) list entries evaluated (up to and including the stop)
    n_blend: np.ndarray    # (P,)
    ambiguous: np.ndarray  # (P,) a decision lies within its margin
    steps: list | None     # per list entry, the forward state needed by the adjoint


def blend(proj, ids: np.ndarray, px: np.ndarray, py: np.ndarray,
          rules: Rules = Rules(), record: bool = False) -> BlendResult:
    """BlendInOrder (Alg. 2) for the pixels (px, py) over the ordered Gaussian list ids."""
    P = px.size
    cxp = px.astype(np.float64) + 0.5
    cyp = py.astype(np.float64) + 0.5
    T = np.ones(P)
    C = np.zeros((P, 3))
    last_pos = np.full(P, -1, np.int64)
    last_id = np.full(P, -1, np.int64)
    done = np.zeros(P, bool)
    n_eval = np.zeros(P, np.int64)
    n_blend = np.zeros(P, np.int64)
    amb = np.zeros(P, bool)
    ext2 = rules.sigma_extent ** 2
    steps = [] if record else None
    for pos, g in enumerate(ids):
        active = ~done
        if not active.any():
            break
        dx = cxp - proj.u[g]
        dy = cyp - proj.v[g]
        Q = proj.conic[g]
        m = Q[0, 0] * dx * dx + 2.0 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
        n_eval += active
        amb |= active & (np.abs(m - ext2) < rules.margin_m * ext2)
        inside = active & (m <= ext2)
        G = np.exp(-0.5 * m)
        raw_alpha = proj.opacity[g] * G
        alpha = np.minimum(rules.alpha_max, raw_alpha)
        amb |= inside & (np.abs(alpha - rules.alpha_min) < rules.margin_alpha * rules.alpha_min)
        take = inside & (alpha >= rules.alpha_min)
        Tn = T * (1.0 - alpha)
        tol = (n_blend + 4) * rules.margin_T_per_step * rules.T_min
        amb |= take & (np.abs(Tn - rules.T_min) < tol)
        stop = take & (Tn < rules.T_min)
        done |= stop
        blended = take & ~stop
        if record:
            steps.append((pos, g, blended.copy(), T.copy(), alpha, G, raw_alpha > rules.alpha_max,
                          dx, dy))
        if blended.any():
            C[blended] += (T * alpha)[blended, None] * proj.rgb[g][None, :]
            T = np.where(blended, Tn, T)
            last_pos[blended] = pos
            last_id[blended] = g
            n_blend += blended
    C += T[:, None] * np.asarray(rules.bg, dtype=np.float64)[None, :]
    return BlendResult(C, T, last_pos, last_id, n_eval, n_blend, amb, steps)


@dataclasses.dataclass
class Image:
    color: np.ndarray       # (H, W, 3)
    T_final: np.ndarray     # (H, W)
    last_id: np.ndarray     # (H, W) Gaussian id of the last blended Gaussian (-1: none)
    n_eval: np.ndarray      # (H, W)
    ambiguous: np.ndarray   # (H, W)
    done: np.ndarray        # (H, W) pixel was rendered by this call


def render_bruteforce(proj, rules: Rules = Rules()) -> Image:
    """Every pixel against every drawable Gaussian in global depth order (no tiles, no AABB)."""
    H, W = proj.height, proj.width
    ids = sort_order(proj, proj.drawable)
    py, px = np.divmod(np.arange(H * W), W)
    r = blend(proj, ids, px, py, rules)
    return Image(r.color.reshape(H, W, 3), r.T_final.reshape(H, W), r.last_id.reshape(H, W),
                 r.n_eval.reshape(H, W), r.ambiguous.reshape(H, W), np.ones((H, W), bool))


def tile_pixels(tile: int, tl: TileLists, width: int, height: int, T: int):
    ty, tx = divmod(tile, tl.tiles_x)
    xs = np.arange(tx * T, min((tx + 1) * T, width))
    ys = np.arange(ty * T, min((ty + 1) * T, height))
    gy, gx = np.meshgrid(ys, xs, indexing="ij")
    return gx.ravel(), gy.ravel()


def render_tiles(proj, rules: Rules = Rules(), tiles=None, tl: TileLists | None = None) -> Image:
    """Alg. 2: per tile, blend the tile's depth-ordered list for each of its pixels.

    ``tiles`` restricts the work to a subset of tile ids (sampled checks at full size).
    """
    H, W = proj.height, proj.width
    tl = tile_lists(proj, rules) if tl is None else tl
    out = Image(np.zeros((H, W, 3)), np.ones((H, W)), np.full((H, W), -1, np.int64),
                np.zeros((H, W), np.int64), np.zeros((H, W), bool), np.zeros((H, W), bool))
    tiles = range(tl.tiles_x * tl.tiles_y) if tiles is None else tiles
    for t in tiles:
        px, py = tile_pixels(int(t), tl, W, H, rules.tile)
        ids = tl.ids[tl.start[t]:tl.start[t + 1]]
        r = blend(proj, ids, px, py, rules)
        out.color[py, px] = r.color
        out.T_final[py, px] = r.T_final
        out.last_id[py, px] = r.last_id
        out.n_eval[py, px] = r.n_eval
        out.ambiguous[py, px] = r.ambiguous
        out.done[py, px] = True
    return out
