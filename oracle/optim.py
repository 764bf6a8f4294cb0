"""The optimiser and schedule of the training loop, in FP64 (oracle side; test
infrastructure only).

Alg. 1 updates every parameter with Adam (Kingma and Ba 2015) from the gradient of
the loss. The textbook update with bias correction, step t >= 1:
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Schedule (Sec. 5.1, Sec. 7.1 implementation details); numbers the paper leaves open
are readings:
* positions: exponential decay of the learning rate (the paper names the technique
  only): log-linear from lr0 to lr1 over the run;
* warm-up: a quarter of the resolution, doubled after iterations 250 and 500;
* SH: degree 0 first, one more band every 1000 iterations up to degree 3;
* density control every 100 iterations after the warm-up (from iteration 500) and
  up to iteration 15000; opacity reset every 3000 iterations.
"""
from __future__ import annotations

import math

import numpy as np


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (returns new p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def position_lr(it, total, lr0, lr1):
    """Log-linear decay from lr0 at iteration 0 to lr1 at iteration `total`."""
    f = min(max(it / max(total, 1), 0.0), 1.0)
    return math.exp((1 - f) * math.log(lr0) + f * math.log(lr1))


def resolution_divisor(it):
    """4 before iteration 250, 2 before 500, then 1."""
    return 4 if it < 250 else (2 if it < 500 else 1)


def sh_degree_at(it, max_degree=3):
    return min(max_degree, it // 1000)


def densify_now(it, start=500, stop=15000, every=100):
    return start <= it <= stop and it % every == 0 and it > 0


def reset_opacity_now(it, every=3000):
    return it > 0 and it % every == 0
