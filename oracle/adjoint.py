"""Analytic reverse-mode derivative of the rasterizer in FP64 (oracle side; test infrastructure only).

Every discrete decision of the forward pass (culls, the 3-sigma test, the alpha
skip, the stop, the alpha clamp, the colour clamp, the order) is held fixed; the
derivative is the exact chain rule through the rest.

Blending (Sec. 6, the back-to-front traversal): with B_i = sum_{j>i} T_j alpha_j c_j
+ T_final bg,
    dC/dc_i = T_i alpha_i,   dC/dalpha_i = T_i c_i - B_i / (1 - alpha_i).
The oracle keeps the forward T_i (it does not recover them by division as the
GPU does), so it also pins that recovery.

alpha = min(0.99, o G), G = exp(-m/2), m = d^T Q d, Q = Sigma'^-1, d = p - (u, v):
    dalpha/do = G and dalpha/dm = -alpha/2 where not clamped, 0 where clamped;
    dm/d(u, v) = -2 Q d;  dm/dQ = d d^T;  dL/dSigma' = -Q (dL/dQ) Q.

Projection (App. A): with U = J W, Sigma' = U Sigma U^T (upper 2x2):
    dL/dSigma = U^T (dL/dSigma') U  (the printed dSigma'/dSigma_ij, contracted),
    dL/dU = 2 (dL/dSigma') U Sigma,  dL/dJ = (dL/dU) W^T;
    dL/dM = 2 (dL/dSigma) M  (dSigma/dM = 2 M^T for symmetric gradients);
    dL/ds_k = sum_i (dL/dM)_ik R_ik  (dM_ij/ds_k = R_ik if j = k);
    dL/dq_hat via the printed matrices dM/dq_r, dM/dq_i, dM/dq_j, dM/dq_k;
    quaternion normalisation: dL/dq = (I - q_hat q_hat^T) / |q| dL/dq_hat;
    activations: dL/dlog s = s dL/ds, dL/dlogit = o (1 - o) dL/do.
The mean receives three terms: through (u, v), through J(t), and through the SH
view direction d = (mu - camera centre) / |mu - camera centre|.
"""
from __future__ import annotations

import numpy as np

from .gaussians import project, sh_basis_grad
from .raster import blend, tile_lists, tile_pixels
from .rules import Rules


def _dM_dq(qh, s):
    """The four printed matrices dM/dq_{r,i,j,k} (App. A), each (N, 3, 3)."""
    r, i, j, k = (qh[:, c] for c in range(4))
    sx, sy, sz = s[:, 0], s[:, 1], s[:, 2]
    z = np.zeros_like(r)

    def mat(rows):
        return 2.0 * np.stack([np.stack(row, -1) for row in rows], 1)
    dr = mat([[z, -sy * k, sz * j], [sx * k, z, -sz * i], [-sx * j, sy * i, z]])
    di = mat([[z, sy * j, sz * k], [sx * j, -2 * sy * i, -sz * r], [sx * k, sy * r, -2 * sz * i]])
    dj = mat([[-2 * sx * j, sy * i, sz * r], [sx * i, z, sz * k], [-sx * r, sy * k, -2 * sz * j]])
    dk = mat([[-2 * sx * k, -sy * r, sz * i], [sx * r, -2 * sy * k, sz * j], [sx * i, sy * j, z]])
    return dr, di, dj, dk


def blend_backward(proj, ids, px, py, dL_dC, rules: Rules, acc: dict):
    """Back-to-front adjoint of one pixel set over one ordered list; accumulates into acc.

    With rules.grad_limit = N > 0 a pixel passes gradient only to its N front-most
    blended Gaussians (the other blended ones still shape the colour behind them).
    """
    fwd = blend(proj, ids, px, py, rules, record=True)
    bg = np.asarray(rules.bg, dtype=np.float64)
    B = fwd.T_final[:, None] * bg[None, :]
    # front-to-back rank of each blended Gaussian at each pixel
    ranks, seen = [], np.zeros(len(px), dtype=np.int64)
    for step in fwd.steps:
        ranks.append(seen.copy())
        seen += step[2]
    for idx in range(len(fwd.steps) - 1, -1, -1):
        pos, g, bl, Tb, alpha, G, clamped, dx, dy = fwd.steps[idx]
        if not bl.any():
            continue
        c = proj.rgb[g]
        gl = bl if rules.grad_limit <= 0 else bl & (ranks[idx] < rules.grad_limit)
        if gl.any():
            gC = dL_dC[gl]                      # (P', 3)
            Ti, ai = Tb[gl], alpha[gl]
            acc["rgb"][g] += (Ti * ai) @ gC
            dalpha = (gC * (Ti[:, None] * c[None, :] - B[gl] / (1.0 - ai)[:, None])).sum(1)
            free = ~clamped[gl]
            if free.any():
                da = dalpha[free]
                acc["opacity"][g] += (da * G[gl][free]).sum()
                dm = da * (-0.5 * ai[free])
                ddx, ddy = dx[gl][free], dy[gl][free]
                Q = proj.conic[g]
                Qdx = Q[0, 0] * ddx + Q[0, 1] * ddy
                Qdy = Q[1, 0] * ddx + Q[1, 1] * ddy
                acc["u"][g] += (dm * (-2.0 * Qdx)).sum()
                acc["v"][g] += (dm * (-2.0 * Qdy)).sum()
                acc["conic"][g] += np.array([[(dm * ddx * ddx).sum(), (dm * ddx * ddy).sum()],
                                             [(dm * ddx * ddy).sum(), (dm * ddy * ddy).sum()]])
        B[bl] += (Tb[bl] * alpha[bl])[:, None] * c[None, :]
    return fwd


def project_backward(scene, proj, g2d: dict) -> dict:
    """Chain rule from the per-Gaussian screen-space gradients to the raw parameters."""
    n = proj.n
    val = proj.valid
    W = proj.W
    Q = proj.conic
    dQ = g2d["conic"]
    dcov = -Q @ dQ @ Q                                    # dL/dSigma'
    U = proj.J @ W
    dSigma = U.transpose(0, 2, 1) @ dcov @ U              # (N, 3, 3)
    dU = 2.0 * dcov @ U @ proj.Sigma                      # (N, 2, 3)
    dJ = dU @ W.T
    tx, ty, tz = proj.t[:, 0], proj.t[:, 1], proj.t[:, 2]
    fx, fy = proj.fx, proj.fy
    du, dv = g2d["u"], g2d["v"]
    dt = np.zeros((n, 3))
    dt[:, 0] = du * fx / tz + dJ[:, 0, 2] * (-fx / (tz * tz))
    dt[:, 1] = dv * fy / tz + dJ[:, 1, 2] * (-fy / (tz * tz))
    dt[:, 2] = (du * (-fx * tx / (tz * tz)) + dv * (-fy * ty / (tz * tz))
                + dJ[:, 0, 0] * (-fx / (tz * tz)) + dJ[:, 0, 2] * (2.0 * fx * tx / tz ** 3)
                + dJ[:, 1, 1] * (-fy / (tz * tz)) + dJ[:, 1, 2] * (2.0 * fy * ty / tz ** 3))
    dmu = dt @ W                                          # dL/dmu_j = sum_r dt_r W_rj
    dM = 2.0 * dSigma @ proj.M
    ds = (dM * proj.R).sum(1)                             # sum_i dM_ik R_ik
    dlog_s = ds * proj.s
    if proj.isotropic:
        # s = exp((l0 + l1 + l2) / 3) on every axis; the quaternion is not used
        dlog_s = np.repeat(dlog_s.sum(1, keepdims=True) / 3.0, 3, 1)
        dq = np.zeros((n, 4))
    else:
        dMq = _dM_dq(proj.qhat, proj.s)
        dqh = np.stack([(dM * d).sum((1, 2)) for d in dMq], 1)
        qh = proj.qhat
        with np.errstate(all="ignore"):
            dq = (dqh - qh * (qh * dqh).sum(1, keepdims=True)) / proj.qnorm[:, None]
    o = proj.opacity
    dlogit = g2d["opacity"] * o * (1.0 - o)
    # colour: only unclamped channels pass gradient
    dc = g2d["rgb"] * (proj.rgb_raw >= 0.0)
    dsh = np.einsum("nk,nc->kcn", proj.shY, dc)
    sh = scene.sh.astype(np.float64)
    gY = sh_basis_grad(proj.sh_degree, proj.dirs)         # (N, K, 3)
    ddir = np.einsum("kcn,nc,nkx->nx", sh, dc, gY)
    d = proj.dirs
    with np.errstate(all="ignore"):
        dmu += (ddir - d * (d * ddir).sum(1, keepdims=True)) / proj.dist[:, None]
    out = {"means": dmu.T, "log_scales": dlog_s.T, "quats": dq.T, "opacity_logits": dlogit,
           "sh": dsh}
    for k, v in out.items():
        v = np.where(val if v.ndim == 1 else (val[None, :] if v.ndim == 2 else val[None, None, :]),
                     v, 0.0)
        out[k] = v
    return out


def empty_acc(n):
    return {"u": np.zeros(n), "v": np.zeros(n), "conic": np.zeros((n, 2, 2)),
            "opacity": np.zeros(n), "rgb": np.zeros((n, 3))}


def render_backward(scene, cam, dL_dC: np.ndarray, rules: Rules = Rules(), tiles=None,
                    bruteforce: bool = False):
    """Forward + analytic backward of one view.

    dL_dC: (H, W, 3) gradient of the loss w.r.t. the rendered image.
    Returns (param_grads, screen_grads, proj). ``tiles`` restricts the pixel set
    (gradients then hold only the contribution of those tiles); ``bruteforce``
    runs every pixel against every drawable Gaussian without tiles.
    """
    proj = project(scene, cam, rules)
    acc = empty_acc(proj.n)
    dL_dC = np.asarray(dL_dC, dtype=np.float64)
    H, W = proj.height, proj.width
    if bruteforce:
        from .raster import sort_order
        ids = sort_order(proj, proj.drawable)
        py, px = np.divmod(np.arange(H * W), W)
        blend_backward(proj, ids, px, py, dL_dC[py, px], rules, acc)
    else:
        tl = tile_lists(proj, rules)
        tiles = range(tl.tiles_x * tl.tiles_y) if tiles is None else tiles
        for t in tiles:
            px, py = tile_pixels(int(t), tl, W, H, rules.tile)
            ids = tl.ids[tl.start[t]:tl.start[t + 1]]
            blend_backward(proj, ids, px, py, dL_dC[py, px], rules, acc)
    return project_backward(scene, proj, acc), acc, proj
