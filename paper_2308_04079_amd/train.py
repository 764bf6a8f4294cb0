"""The optimisation loop of Alg. 1 on the HIP kernels: render, photometric loss
(Sec. 5.1), backward, Adam, and adaptive density control (Sec. 5.2) on the
schedule of Sec. 5.1 and Sec. 7.1.

Schedule (numbers the paper leaves open are readings, each a field of TrainConfig):
* positions: the learning rate decays log-linearly from lr_means[0] to
  lr_means[1] (times the scene extent) over the run; every other group is constant,
  covariance (log-scales, quaternions) at the paper's 0.001;
* warm-up: a quarter of the resolution, doubled after iterations 250 and 500;
* SH: degree 0 first, one band more every 1000 iterations;
* density control every 100 iterations from 500 to 15000, opacity reset every 3000;
  the optimiser moments of kept Gaussians are carried over, those of clones and
  split children start at zero.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import types

import numpy as np
import torch

from . import _lib
from .density import DensityControl, reset_opacity
from .raster import GaussianParams, Rasterizer, RenderState, photometric_loss_grad

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


@dataclasses.dataclass
class TrainConfig:
    iterations: int = 30000
    views_per_step: int = 1
    lam: float = 0.2                            # D-SSIM weight (Sec. 5.1)
    lr_means: tuple = (1.6e-4, 1.6e-6)          # x scene extent, decayed log-linearly
    lr_log_scales: float = 1e-3                 # covariance (Sec. 7.1)
    lr_quats: float = 1e-3
    lr_opacity: float = 0.05
    lr_sh_dc: float = 2.5e-3
    lr_sh_rest: float = 2.5e-3 / 20
    betas: tuple = (0.9, 0.999)
    eps: float = 1e-15
    warmup: tuple = (250, 500)                  # resolution /4 before, /2 between, /1 after
    sh_every: int = 1000                        # <= 0: every band from the start
    densify_from: int = 500
    densify_until: int = 15000
    densify_every: int = 100
    reset_every: int = 3000
    split_fraction: float = 0.01                # split above this fraction of the extent
    max_world_fraction: float = 0.1             # remove above this fraction (after a reset)
    max_screen_radius: float = 20.0             # remove above this pixel radius (after a reset)
    seed: int = 0


def scaled_camera(cam, div: int):
    """The same view at 1/div of the resolution (pixel centres keep their meaning)."""
    if div == 1:
        return cam
    return types.SimpleNamespace(R=cam.R, t=cam.t, fx=np.float32(cam.fx / div),
                                 fy=np.float32(cam.fy / div), cx=np.float32(cam.cx / div),
                                 cy=np.float32(cam.cy / div), width=max(1, cam.width // div),
                                 height=max(1, cam.height // div))


def downsample(img: torch.Tensor, cam, div: int) -> torch.Tensor:
    """Box-filter a planar [3][H][W] image by div (the warm-up targets)."""
    if div == 1:
        return img.reshape(-1)
    h, w = cam.height // div, cam.width // div
    x = img.view(3, cam.height, cam.width)[:, :h * div, :w * div]
    return x.reshape(3, h, div, w, div).mean(dim=(2, 4)).contiguous().reshape(-1)


class Trainer:
    """Owns the parameters, the Adam moments and the density statistics."""

    def __init__(self, params: GaussianParams, cams, targets, extent: float,
                 cfg: TrainConfig | None = None, max_sh_degree: int | None = None):
        self.cfg = cfg if cfg is not None else TrainConfig()
        cfg = self.cfg
        self.params = params
        self.cams = list(cams)
        self.extent = float(extent)
        self.max_deg = params.sh_degree if max_sh_degree is None else max_sh_degree
        self.targets = {1: [t.reshape(-1) for t in targets]}
        for div in (2, 4):
            self.targets[div] = [downsample(t, c, div) for t, c in zip(targets, self.cams)]
        self.m = self._zeros_like(params)
        self.v = self._zeros_like(params)
        self.t = 0
        self.it = 0
        self.rng = np.random.default_rng(cfg.seed)
        self.rasts = {}
        self.capacity = None
        self.dc = DensityControl(params.n, params.means.device,
                                 split_scale=cfg.split_fraction * self.extent)
        self.history = []

    @staticmethod
    def _zeros_like(p: GaussianParams) -> GaussianParams:
        return GaussianParams(*(torch.zeros_like(getattr(p, k)) for k in GROUPS))

    # -- schedule ------------------------------------------------------------------
    def resolution_divisor(self, it):
        a, b = self.cfg.warmup
        return 4 if it < a else (2 if it < b else 1)

    def sh_degree(self, it):
        if self.cfg.sh_every <= 0:
            return self.max_deg
        return min(self.max_deg, it // self.cfg.sh_every)

    def lr_means(self, it):
        f = min(max(it / max(self.cfg.iterations, 1), 0.0), 1.0)
        l0, l1 = self.cfg.lr_means
        return self.extent * math.exp((1 - f) * math.log(l0) + f * math.log(l1))

    def densify_now(self, it):
        c = self.cfg
        return c.densify_from <= it <= c.densify_until and it > 0 and it % c.densify_every == 0

    def reset_now(self, it):
        return it > 0 and it % self.cfg.reset_every == 0

    def _rasterizer(self, deg):
        if deg not in self.rasts:
            self.rasts[deg] = Rasterizer(sh_degree=deg, capacity=self.capacity)
        r = self.rasts[deg]
        if self.capacity is not None and (r.capacity is None or r.capacity < self.capacity):
            r.capacity = self.capacity
        return r

    # -- one iteration -------------------------------------------------------------
    def step(self):
        cfg, it = self.cfg, self.it
        idx = self.rng.choice(len(self.cams), cfg.views_per_step, replace=False)
        div = self.resolution_divisor(it)
        cams = [scaled_camera(self.cams[i], div) for i in idx]
        target = torch.cat([self.targets[div][i] for i in idx])
        rast = self._rasterizer(self.sh_degree(it))
        state = rast.render(self.params, cams)
        self.capacity = max(self.capacity or 0, rast.capacity)
        loss = torch.zeros(len(cams), dtype=torch.float32, device=target.device)
        dL = photometric_loss_grad(state, target, cfg.lam, loss)
        grads, grad2d = rast.backward(self.params, state, dL)
        if it <= cfg.densify_until:
            self.dc.accumulate(state, grad2d)
        self._adam(grads, it)
        self.it += 1
        it = self.it
        if self.densify_now(it):
            self._densify(prune_large=it > cfg.reset_every)
        if self.reset_now(it):
            reset_opacity(self.params.opacity_logits, 0.01)
        self.history.append(loss)
        return loss

    def _adam(self, grads, it):
        cfg = self.cfg
        self.t += 1
        lr = {"means": self.lr_means(it), "log_scales": cfg.lr_log_scales,
              "quats": cfg.lr_quats, "opacity_logits": cfg.lr_opacity}
        lib = _lib.lib()
        stream = torch.cuda.current_stream(self.params.means.device).cuda_stream
        b1, b2 = cfg.betas

        def run(p, g, m, v, rate):
            _lib.check("gs_adam_step", lib.gs_adam_step(
                _lib.ptr(p), _lib.ptr(g), _lib.ptr(m), _lib.ptr(v), p.numel(), float(rate),
                float(b1), float(b2), float(cfg.eps), self.t, stream))
        for k, rate in lr.items():
            run(getattr(self.params, k), grads[k], getattr(self.m, k), getattr(self.v, k), rate)
        # SH: the DC plane and the higher bands take different rates. Bands the ramp has
        # not reached yet have zero gradients and still-zero moments, on which an Adam
        # step changes nothing (m = v = 0, update 0 / eps = 0): they are skipped.
        sh, g = self.params.sh, grads["sh"]
        run(sh[0], g[0], self.m.sh[0], self.v.sh[0], cfg.lr_sh_dc)
        k_active = min(sh.shape[0], (self.sh_degree(it) + 1) ** 2)
        if k_active > 1:
            run(sh[1:k_active], g[1:k_active], self.m.sh[1:k_active], self.v.sh[1:k_active],
                cfg.lr_sh_rest)

    def _densify(self, prune_large: bool):
        cfg = self.cfg
        dc = self.dc
        dc.cfg.max_world_scale = cfg.max_world_fraction * self.extent if prune_large else 0.0
        dc.cfg.max_screen_radius = cfg.max_screen_radius if prune_large else 0.0
        action, offsets, n_new = dc.plan(self.params)
        new, _ = dc.apply(self.params, action, offsets, n_new)
        deg = self.params.sh_degree
        lib = _lib.lib()
        stream = torch.cuda.current_stream(self.params.means.device).cuda_stream
        moments = []
        for st in (self.m, self.v):
            out = self._empty(n_new, st.sh.shape[0], st.means.device)
            if n_new > 0:
                src = st.c_struct()
                dst = _lib.GsParamsGrad(*(_lib.ptr(getattr(out, k)) for k in GROUPS))
                _lib.check("gs_densify_gather", lib.gs_densify_gather(
                    ctypes.byref(src), deg, _lib.ptr(action), _lib.ptr(offsets), 1,
                    ctypes.byref(dst), n_new, stream))
            moments.append(out)
        self.params, (self.m, self.v) = new, moments
        dc.reset_stats(n_new)

    @staticmethod
    def _empty(n, K, dev):
        return GaussianParams(torch.empty(3, n, device=dev), torch.empty(3, n, device=dev),
                              torch.empty(4, n, device=dev), torch.empty(n, device=dev),
                              torch.empty(K, 3, n, device=dev))


__all__ = ["TrainConfig", "Trainer", "scaled_camera", "downsample", "RenderState"]
