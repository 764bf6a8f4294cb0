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

from .rules import EPS32, Rules


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
    ambiguous: np.ndarray  # (P,) a decision that shapes the image lies within its margin
    ambiguous_grad: np.ndarray  # (P,) ambiguous, or an alpha-clamp decision within its margin
    T_err: np.ndarray      # (P,) bound on the relative FP32 rounding error of T_final
    steps: list | None     # per list entry, the forward state needed by the adjoint
    flags: list | None     # per pixel, the (position, kind) of every decision within its margin


# kinds of threshold decision, in the order an entry takes them
DECIDE_EXTENT, DECIDE_ALPHA, DECIDE_STOP = 0, 1, 2


def _whitening(proj, g):
    """The whitening factor L^-1 = [[w00, 0], [w10, w11]] of Sigma' = L L^T (lower
    Cholesky factor L), so that m = |L^-1 d|^2."""
    a, b, c = proj.cov2d[g, 0, 0], proj.cov2d[g, 0, 1], proj.cov2d[g, 1, 1]
    l00 = np.sqrt(a)
    l10 = b / l00
    l11 = np.sqrt(max(c - l10 * l10, 0.0))
    return 1.0 / l00, -l10 / (l00 * l11), 1.0 / l11


def _f32_gap(x: float) -> float:
    """Distance between a threshold and its FP32 representation."""
    return abs(float(np.float32(x)) - x)


def blend(proj, ids: np.ndarray, px: np.ndarray, py: np.ndarray,
          rules: Rules = Rules(), record: bool = False, forced=frozenset(),
          flags: bool = False) -> BlendResult:
    """BlendInOrder (Alg. 2) for the pixels (px, py) over the ordered Gaussian list ids.

    ``forced`` holds (list position, decision kind) pairs whose decision is taken
    the other way at every pixel of the call (the legitimate alternative outcomes
    of a decision within its margin); ``flags`` records, per pixel, every decision
    that lies within its margin.
    """
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
    amb_grad = np.zeros(P, bool)
    T_err = np.zeros(P)          # relative error bound of the running T
    ext2 = rules.sigma_extent ** 2
    Km, Ka, Kt, eps = rules.margin_m, rules.margin_alpha, rules.margin_T, EPS32
    gap_amin, gap_amax, gap_Tmin = (_f32_gap(rules.alpha_min), _f32_gap(rules.alpha_max),
                                    _f32_gap(rules.T_min))
    steps = [] if record else None
    flag_list = [[] for _ in range(P)] if flags else None
    for pos, g in enumerate(ids):
        active = ~done
        if not active.any():
            break
        dx = cxp - proj.u[g]
        dy = cyp - proj.v[g]
        Q = proj.conic[g]
        m = Q[0, 0] * dx * dx + 2.0 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
        n_eval += active
        # FP32 error bound of m evaluated as |L^-1 D + c|^2: D = pixel centre minus the
        # centre of the box's corner pixel (exact), c = L^-1 (corner centre - mean) and
        # L^-1 rounded to FP32, then two fused multiply-adds per component
        w00, w10, w11 = _whitening(proj, g)
        ax, ay = (proj.i_lo[g] + 0.5) - proj.u[g], (proj.j_lo[g] + 0.5) - proj.v[g]
        c0, c1 = w00 * ax, w10 * ax + w11 * ay
        Di = np.abs(px - proj.i_lo[g]).astype(np.float64)
        Dj = np.abs(py - proj.j_lo[g]).astype(np.float64)
        e0 = np.abs(w00 * dx)
        e1 = np.sqrt(np.maximum(m - e0 * e0, 0.0))
        inner = np.abs(w11 * (py - proj.j_lo[g]) + c1)
        de0 = eps * (abs(w00) * Di + abs(c0) + e0)
        de1 = eps * (abs(w10) * Di + abs(w11) * Dj + abs(c1) + inner + e1)
        err_m = 2.0 * (e0 * de0 + e1 * de1) + eps * (e1 * e1 + m)
        G = np.exp(-0.5 * m)
        raw_alpha = proj.opacity[g] * G
        clamped = raw_alpha > rules.alpha_max
        alpha = np.minimum(rules.alpha_max, raw_alpha)
        rel_a = np.where(clamped, eps, 0.5 * err_m + eps * (m + 8.0))

        flip = [(pos, k) in forced for k in (DECIDE_EXTENT, DECIDE_ALPHA, DECIDE_STOP)]
        near_m = active & (np.abs(m - ext2) < Km * err_m)
        inside = active & ((m <= ext2) != flip[0])
        near_a = inside & (np.abs(alpha - rules.alpha_min) < Ka * (rel_a * alpha + gap_amin))
        take = inside & ((alpha >= rules.alpha_min) != flip[1])
        Tn = T * (1.0 - alpha)
        rel_Tn = T_err + alpha / (1.0 - alpha) * rel_a + 2.0 * eps
        near_s = take & (np.abs(Tn - rules.T_min) < Kt * (rel_Tn * Tn + gap_Tmin))
        stop = take & ((Tn < rules.T_min) != flip[2])
        near_c = take & (np.abs(raw_alpha - rules.alpha_max) <
                         Ka * ((0.5 * err_m + eps * (m + 8.0)) * raw_alpha + gap_amax))
        amb |= near_m | near_a | near_s
        amb_grad |= near_m | near_a | near_s | near_c
        if flags:
            for k, near in ((DECIDE_EXTENT, near_m), (DECIDE_ALPHA, near_a), (DECIDE_STOP, near_s)):
                for p_ in np.nonzero(near)[0]:
                    flag_list[p_].append((pos, k))
        done |= stop
        blended = take & ~stop
        if record:
            steps.append((pos, g, blended.copy(), T.copy(), alpha, G, clamped, dx, dy))
        if blended.any():
            C[blended] += (T * alpha)[blended, None] * proj.rgb[g][None, :]
            T = np.where(blended, Tn, T)
            T_err = np.where(blended, rel_Tn, T_err)
            last_pos[blended] = pos
            last_id[blended] = g
            n_blend += blended
    C += T[:, None] * np.asarray(rules.bg, dtype=np.float64)[None, :]
    return BlendResult(C, T, last_pos, last_id, n_eval, n_blend, amb, amb_grad, T_err, steps,
                       flag_list)


def pixel_outcomes(proj, ids: np.ndarray, x: int, y: int, rules: Rules = Rules(),
                   limit: int = 64) -> list:
    """Every legitimate outcome of one pixel: the blend with each combination of its
    within-margin decisions taken either way (depth first, at most ``limit`` runs).

    A decision ahead of every forced one is the same in every run, so each branch
    only flips decisions that come after the last one it already forced.
    """
    px, py = np.array([x]), np.array([y])
    out = []

    def explore(forced: tuple):
        r = blend(proj, ids, px, py, rules, forced=frozenset(forced), flags=True)
        out.append(r)
        after = forced[-1] if forced else (-1, -1)
        for d in r.flags[0]:
            if len(out) >= limit:
                return
            if d > after:
                explore(forced + (d,))

    explore(())
    return out


@dataclasses.dataclass
class Image:
    color: np.ndarray       # (H, W, 3)
    T_final: np.ndarray     # (H, W)
    last_id: np.ndarray     # (H, W) Gaussian id of the last blended Gaussian (-1: none)
    n_eval: np.ndarray      # (H, W)
    ambiguous: np.ndarray   # (H, W)
    done: np.ndarray        # (H, W) pixel was rendered by this call
    ambiguous_grad: np.ndarray  # (H, W) ambiguous, or an alpha clamp within its margin
    T_err: np.ndarray       # (H, W) relative FP32 error bound of T_final


def render_bruteforce(proj, rules: Rules = Rules()) -> Image:
    """Every pixel against every drawable Gaussian in global depth order (no tiles, no AABB)."""
    H, W = proj.height, proj.width
    ids = sort_order(proj, proj.drawable)
    py, px = np.divmod(np.arange(H * W), W)
    r = blend(proj, ids, px, py, rules)
    return Image(r.color.reshape(H, W, 3), r.T_final.reshape(H, W), r.last_id.reshape(H, W),
                 r.n_eval.reshape(H, W), r.ambiguous.reshape(H, W), np.ones((H, W), bool),
                 r.ambiguous_grad.reshape(H, W), r.T_err.reshape(H, W))


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
                np.zeros((H, W), np.int64), np.zeros((H, W), bool), np.zeros((H, W), bool),
                np.zeros((H, W), bool), np.zeros((H, W)))
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
        out.ambiguous_grad[py, px] = r.ambiguous_grad
        out.T_err[py, px] = r.T_err
        out.done[py, px] = True
    return out
