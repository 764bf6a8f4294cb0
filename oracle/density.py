"""Adaptive density control in FP64 (oracle side; test infrastructure only).

Sec. 5.2 and Alg. 1: every 100 iterations, Gaussians that are essentially
transparent (alpha below epsilon_alpha) or too large are removed; Gaussians whose
average view-space positional gradient exceeds tau_pos = 0.0002 are densified:
small ones are cloned (a copy of the same size), large ones are split into two
whose scale is the original divided by phi = 1.6 and whose positions are sampled
with the original Gaussian as the PDF. Every 3000 iterations the opacities are
set close to zero.

Readings where the paper gives no number or leaves the quantity open:
* the view-space positional gradient is the gradient of the loss with respect to
  the projected mean in normalised device coordinates (x_ndc = 2u/W - 1), so its
  norm per view is |(W/2 dL/du, H/2 dL/dv)|; its average is over the views in which
  the Gaussian was visible since the statistics were reset;
* epsilon_alpha = 0.005; "large" for split versus clone means a largest scale
  above split_scale (a fraction of the scene extent chosen by the caller);
  "too large" means a largest scale above max_world_scale or a pixel-box
  half-extent above max_screen_radius (either test disabled when <= 0);
* a clone is an exact copy (the next optimiser step moves it along the gradient);
* the two split children are mu + R diag(s) z with z ~ N(0, I) drawn per child,
  the original is removed; the opacity reset caps alpha at 0.01.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .gaussians import quaternion_to_rotation

REMOVE, KEEP, CLONE, SPLIT = 0, 1, 2, 3


@dataclasses.dataclass(frozen=True)
class DensifyRules:
    grad_threshold: float = 0.0002
    min_opacity: float = 0.005
    split_scale: float = 0.01
    max_world_scale: float = 0.0
    max_screen_radius: float = 0.0
    split_factor: float = 1.6


def accumulate(du, dv, visible, widths, heights):
    """Per-view screen gradients (V, N) -> (sum of NDC gradient norms, visible-view count)."""
    du = np.asarray(du, dtype=np.float64)
    dv = np.asarray(dv, dtype=np.float64)
    w = np.asarray(widths, dtype=np.float64)[:, None] / 2.0
    h = np.asarray(heights, dtype=np.float64)[:, None] / 2.0
    norm = np.sqrt((du * w) ** 2 + (dv * h) ** 2)
    return (norm * visible).sum(0), visible.sum(0).astype(np.int64)


def screen_radius(i_lo, i_hi, j_lo, j_hi):
    """Half the larger side, in pixels, of an inclusive pixel box (the 2D size test)."""
    w = np.asarray(i_hi, np.int64) - np.asarray(i_lo, np.int64) + 1
    h = np.asarray(j_hi, np.int64) - np.asarray(j_lo, np.int64) + 1
    return 0.5 * np.maximum(w, h)


def plan(scene, grad_sum, view_count, max_radius, rules: DensifyRules = DensifyRules()):
    """The action of every Gaussian (Alg. 1) and its number of output Gaussians."""
    logit = scene.opacity_logits.astype(np.float64)
    o = 1.0 / (1.0 + np.exp(-logit))
    smax = np.exp(scene.log_scales.astype(np.float64).max(0))
    avg = np.where(view_count > 0, grad_sum / np.maximum(view_count, 1), 0.0)
    too_large = np.zeros(scene.n, bool)
    if rules.max_world_scale > 0:
        too_large |= smax > rules.max_world_scale
    if rules.max_screen_radius > 0:
        too_large |= max_radius > rules.max_screen_radius
    remove = (o < rules.min_opacity) | too_large
    densify = ~remove & (avg > rules.grad_threshold)
    split = densify & (smax > rules.split_scale)
    clone = densify & ~split
    action = np.full(scene.n, KEEP, np.int64)
    action[remove] = REMOVE
    action[clone] = CLONE
    action[split] = SPLIT
    out_count = np.array([0, 1, 2, 2])[action]
    return action, out_count


def apply(scene, action, normals, rules: DensifyRules = DensifyRules()):
    """New parameter arrays (FP64) in Gaussian order; normals (N, 2, 3) feed the splits."""
    mu = scene.means.astype(np.float64).T
    ls = scene.log_scales.astype(np.float64).T
    q = scene.quats.astype(np.float64).T
    lg = scene.opacity_logits.astype(np.float64)
    sh = scene.sh.astype(np.float64)
    out = {k: [] for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "src")}
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    R = quaternion_to_rotation(qn)
    s = np.exp(ls)
    for g in range(scene.n):
        a = action[g]
        if a == REMOVE:
            continue
        copies = 1 if a == KEEP else 2
        for c in range(copies):
            if a == SPLIT:
                out["means"].append(mu[g] + R[g] @ (s[g] * normals[g, c]))
                out["log_scales"].append(ls[g] - np.log(rules.split_factor))
            else:
                out["means"].append(mu[g])
                out["log_scales"].append(ls[g])
            out["quats"].append(q[g])
            out["opacity_logits"].append(lg[g])
            out["sh"].append(sh[:, :, g])
            out["src"].append(g)
    res = {k: np.array(v) for k, v in out.items()}
    return res


def reset_opacity(logits, max_opacity=0.01):
    """Opacity reset: alpha <- min(alpha, max_opacity), in logit space."""
    cap = np.log(max_opacity / (1.0 - max_opacity))
    return np.minimum(np.asarray(logits, dtype=np.float64), cap)
