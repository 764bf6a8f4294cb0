"""Adaptive density control driver (Sec. 5.2, Alg. 1): statistics, plan, apply, reset.

Argument marshalling over the gs_densify_* entry points of libgs_mi355x.so; the
only host synchronisation is reading the new Gaussian count, once per
densification (every 100 iterations in the paper).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .raster import GaussianParams, RenderState

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


class DensityControl:
    def __init__(self, n: int, device="cuda", **overrides):
        self.cfg = _lib.GsDensifyConfig()
        _lib.lib().gs_default_densify_config(ctypes.byref(self.cfg))
        for k, v in overrides.items():
            setattr(self.cfg, k, float(v))
        self.device = torch.device(device)
        self.reset_stats(n)

    def reset_stats(self, n: int):
        self.n = n
        self.grad_sum = torch.zeros(max(n, 1), dtype=torch.float32, device=self.device)
        self.view_count = torch.zeros(max(n, 1), dtype=torch.int32, device=self.device)
        self.max_radius = torch.zeros(max(n, 1), dtype=torch.float32, device=self.device)

    def accumulate(self, state: RenderState, grad2d: torch.Tensor):
        """Add one backward pass's positional-gradient statistics."""
        self.accumulate_raw(state.projected(), state.cams_c, state.n_views, state.n, grad2d)

    def accumulate_raw(self, proj, cams_c, n_views: int, n: int, grad2d: torch.Tensor):
        if n != self.n:
            raise ValueError("statistics were sized for a different Gaussian count")
        if grad2d.dtype != torch.float32 or grad2d.numel() < n_views * n * _lib.GRAD2D_FLOATS:
            raise ValueError("grad2d must be float32 [V*N][9]")
        _lib.check("gs_densify_accumulate", _lib.lib().gs_densify_accumulate(
            ctypes.byref(proj), _lib.ptr(grad2d), cams_c, n_views, n,
            _lib.ptr(self.grad_sum), _lib.ptr(self.view_count), _lib.ptr(self.max_radius),
            torch.cuda.current_stream(self.device).cuda_stream))

    def plan(self, params: GaussianParams):
        """(action uint8 [N], offsets int32 [N], new count)."""
        lib = _lib.lib()
        n = params.n
        stream = torch.cuda.current_stream(self.device).cuda_stream
        action = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        offsets = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        n_out = torch.zeros(1, dtype=torch.int32, device=self.device)
        ws = torch.empty(max(1, lib.gs_densify_workspace_bytes(n)), dtype=torch.uint8,
                         device=self.device)
        pr = params.c_struct()
        _lib.check("gs_densify_plan", lib.gs_densify_plan(
            ctypes.byref(pr), _lib.ptr(self.grad_sum), _lib.ptr(self.view_count),
            _lib.ptr(self.max_radius), ctypes.byref(self.cfg), _lib.ptr(action),
            _lib.ptr(offsets), _lib.ptr(n_out), _lib.ptr(ws), ws.numel(), stream))
        return action, offsets, int(n_out.item())

    def apply(self, params: GaussianParams, action, offsets, n_new: int,
              normals: torch.Tensor | None = None, generator: torch.Generator | None = None):
        """New parameters and, per new Gaussian, its source index."""
        n = params.n
        K = params.sh.shape[0]
        if n_new == 0:
            e = lambda *shape: torch.empty(*shape, device=self.device)  # noqa: E731
            return (GaussianParams(e(3, 0), e(3, 0), e(4, 0), e(0), e(K, 3, 0)),
                    torch.empty(0, dtype=torch.int32, device=self.device))
        if normals is None:
            normals = torch.randn(max(n, 1), 2, 3, device=self.device, generator=generator)
        normals = normals.contiguous().float()
        if normals.numel() < n * 6:
            raise ValueError("normals must hold [N][2][3] values")
        out = GaussianParams(
            torch.empty(3, n_new, device=self.device), torch.empty(3, n_new, device=self.device),
            torch.empty(4, n_new, device=self.device), torch.empty(n_new, device=self.device),
            torch.empty(K, 3, n_new, device=self.device))
        src = torch.empty(max(n_new, 1), dtype=torch.int32, device=self.device)
        gp = _lib.GsParamsGrad(*(_lib.ptr(getattr(out, k)) for k in GROUPS))
        pr = params.c_struct()
        _lib.check("gs_densify_apply", _lib.lib().gs_densify_apply(
            ctypes.byref(pr), params.sh_degree, _lib.ptr(action), _lib.ptr(offsets),
            _lib.ptr(normals), ctypes.byref(self.cfg), ctypes.byref(gp), n_new, _lib.ptr(src),
            torch.cuda.current_stream(self.device).cuda_stream))
        return out, src[:n_new]

    def densify(self, params: GaussianParams, normals=None, generator=None):
        """Plan and apply, then reset the statistics for the new count."""
        action, offsets, n_new = self.plan(params)
        out, src = self.apply(params, action, offsets, n_new, normals, generator)
        self.reset_stats(n_new)
        return out, src, action


def reset_opacity(opacity_logits: torch.Tensor, max_opacity: float = 0.01):
    """In place: opacity <- min(opacity, max_opacity) (the periodic reset of Sec. 5.2)."""
    _lib.check("gs_reset_opacity", _lib.lib().gs_reset_opacity(
        _lib.ptr(opacity_logits), opacity_logits.numel(), float(max_opacity),
        torch.cuda.current_stream(opacity_logits.device).cuda_stream))
