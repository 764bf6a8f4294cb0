"""Python driver of the HIP rasterizer: buffers (torch device memory), streams, autograd.

Argument marshalling only: every step of the forward and backward pass runs in
libgs_mi355x.so. The stages follow Alg. 2 of Kerbl et al. (2023):
gs_project -> gs_bin -> gs_sort -> gs_render_fwd, and backward
gs_render_bwd -> gs_project_bwd (Sec. 6, App. A).
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib


@dataclasses.dataclass
class GaussianParams:
    """Raw Gaussian parameters, SoA float32 on the GPU (see include/gs.h for layouts)."""
    means: torch.Tensor           # (3, N)
    log_scales: torch.Tensor      # (3, N)
    quats: torch.Tensor           # (4, N)
    opacity_logits: torch.Tensor  # (N,)
    sh: torch.Tensor              # (K, 3, N)

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def sh_degree(self) -> int:
        return int(round(self.sh.shape[0] ** 0.5)) - 1

    def c_struct(self) -> _lib.GsParams:
        for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            t = getattr(self, name)
            if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError(f"{name} must be a contiguous float32 GPU tensor")
        return _lib.GsParams(_lib.ptr(self.means), _lib.ptr(self.log_scales), _lib.ptr(self.quats),
                             _lib.ptr(self.opacity_logits), _lib.ptr(self.sh), self.n)

    @staticmethod
    def from_numpy(scene, device="cuda") -> "GaussianParams":
        def t(a):
            return torch.from_numpy(a.astype("float32", copy=False)).contiguous().to(device)
        return GaussianParams(t(scene.means), t(scene.log_scales), t(scene.quats),
                              t(scene.opacity_logits), t(scene.sh))


@dataclasses.dataclass
class RenderState:
    """Everything the forward pass leaves for the backward pass (and for inspection)."""
    n: int
    cams: list
    cams_c: ctypes.Array
    n_views: int
    n_tiles: int
    tile_offset: list
    pix_offset: list
    depth_key: torch.Tensor
    tiles_touched: torch.Tensor
    record: torch.Tensor
    keys: torch.Tensor
    vals: torch.Tensor
    keys_alt: torch.Tensor
    vals_alt: torch.Tensor
    count: torch.Tensor
    status: torch.Tensor
    capacity: int
    ranges: torch.Tensor
    order: torch.Tensor       # tile issue order (longest list first)
    image: torch.Tensor       # flat: per view [3][H][W] at 3 * pix_offset[v]
    T_final: torch.Tensor     # flat: per view [H][W] at pix_offset[v]
    last_idx: torch.Tensor

    def projected(self) -> _lib.GsProjected:
        return _lib.GsProjected(_lib.ptr(self.depth_key), _lib.ptr(self.tiles_touched),
                                _lib.ptr(self.record))

    def instances(self) -> _lib.GsInstances:
        return _lib.GsInstances(_lib.ptr(self.keys), _lib.ptr(self.vals), _lib.ptr(self.keys_alt),
                                _lib.ptr(self.vals_alt), self.capacity, _lib.ptr(self.count),
                                _lib.ptr(self.status))

    def tile_ids(self, cfg) -> torch.Tensor:
        """Sorted global tile id of every instance (int32 view of the scratch buffer)."""
        inst = self.instances()
        addr = _lib.lib().gs_sorted_tile_ids(ctypes.byref(inst), self.n_tiles, ctypes.byref(cfg))
        if not addr:
            raise _lib.GsError("gs_sorted_tile_ids", _lib.ERR_ARG)
        for buf in (self.keys, self.keys_alt):
            words = buf.view(torch.int32)
            off = (addr - buf.data_ptr()) // 4
            if 0 <= off < words.numel():
                return words[off:off + self.capacity]
        raise RuntimeError("sorted tile ids outside the instance buffers")

    def view_image(self, v: int) -> torch.Tensor:
        c = self.cams[v]
        p = self.pix_offset[v]
        return self.image[3 * p:3 * (p + c.width * c.height)].view(3, c.height, c.width)

    def view_plane(self, buf: torch.Tensor, v: int) -> torch.Tensor:
        c = self.cams[v]
        p = self.pix_offset[v]
        return buf[p:p + c.width * c.height].view(c.height, c.width)

    def read_status(self):
        """(status bits, instance count); synchronises the current stream."""
        st, ct = ctypes.c_uint32(0), ctypes.c_uint32(0)
        inst = self.instances()
        _lib.lib().gs_read_status(ctypes.byref(inst), ctypes.byref(st), ctypes.byref(ct),
                                  torch.cuda.current_stream(self.status.device).cuda_stream)
        return int(st.value), int(ct.value)


class Rasterizer:
    """Forward and backward of the tile rasterizer over V >= 1 views per call.

    capacity: instance capacity (grows automatically when ``check`` is on).
    isotropic, grad_limit: the ablation switches of Sec. 7.3 (see gs_config).
    """

    def __init__(self, sh_degree: int = 3, tile_size: int = 16, bg=(0.0, 0.0, 0.0),
                 capacity: int | None = None, growth: float = 1.25, sort_digit_bits: int = 8,
                 lds_batch: int = 64, isotropic: bool = False, grad_limit: int = 0):
        self.cfg = _lib.default_config(sh_degree=sh_degree, tile_size=tile_size, bg=bg,
                                       sort_digit_bits=sort_digit_bits, lds_batch=lds_batch,
                                       isotropic=int(bool(isotropic)), grad_limit=int(grad_limit))
        self.capacity = capacity
        self.growth = growth
        self.check = True   # RasterizeFunction: read the status word after each forward

    # -- forward -----------------------------------------------------------------
    def render(self, params: GaussianParams, cams, check: bool = True,
               for_backward: bool = True) -> RenderState:
        """Project, bin, sort and blend all views. ``for_backward=False`` is the
        forward-only path: no per-pixel backward state is written (T_final and
        last_idx of the result are empty)."""
        lib = _lib.lib()
        if params.sh_degree < self.cfg.sh_degree:
            raise ValueError(f"params carry SH degree {params.sh_degree}, config has "
                             f"{self.cfg.sh_degree}")
        # a higher stored degree renders its first (deg + 1)^2 bands (the SH ramp)
        cams = list(cams)
        V = len(cams)
        n = params.n
        dev = params.means.device
        stream = torch.cuda.current_stream(dev).cuda_stream
        cams_c = _lib.make_cameras(cams)
        cfg = ctypes.byref(self.cfg)
        toff = (ctypes.c_int64 * (V + 1))()
        n_tiles = lib.gs_tile_layout(cams_c, V, self.cfg.tile_size, toff)
        _lib.check("gs_tile_layout", 0 if n_tiles > 0 else int(n_tiles))
        pix = [0]
        for c in cams:
            pix.append(pix[-1] + int(c.width) * int(c.height))

        depth_key = torch.empty(max(1, V * n), dtype=torch.int32, device=dev)
        tiles_touched = torch.empty(max(1, V * n), dtype=torch.int32, device=dev)  # gs_project writes all
        record = torch.empty(max(1, V * n) * _lib.RECORD_FLOATS, dtype=torch.float32, device=dev)
        pr = params.c_struct()
        proj = _lib.GsProjected(_lib.ptr(depth_key), _lib.ptr(tiles_touched), _lib.ptr(record))
        _lib.check("gs_project", lib.gs_project(ctypes.byref(pr), cams_c, V, cfg,
                                                ctypes.byref(proj), stream))
        cap = self.capacity if self.capacity is not None else max(1 << 16, 2 * n * V)
        ranges = torch.empty(2 * n_tiles, dtype=torch.int32, device=dev)
        order = torch.empty(n_tiles, dtype=torch.int32, device=dev)
        image = torch.empty(3 * pix[-1], dtype=torch.float32, device=dev)
        npix = pix[-1] if for_backward else 0
        T_final = torch.empty(npix, dtype=torch.float32, device=dev)
        last_idx = torch.empty(npix, dtype=torch.int32, device=dev)
        bin_ws = torch.empty(max(1, lib.gs_bin_workspace_bytes(V * n, cfg)), dtype=torch.uint8,
                             device=dev)
        while True:
            cap = min(int(cap), _lib.MAX_INSTANCES)
            keys = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
            vals = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            keys_alt = torch.empty_like(keys)
            vals_alt = torch.empty_like(vals)
            words = torch.zeros(2, dtype=torch.int32, device=dev)   # one fill for both
            count, status = words[0:1], words[1:2]
            state = RenderState(n, cams, cams_c, V, int(n_tiles), list(toff), pix, depth_key,
                                tiles_touched, record, keys, vals, keys_alt, vals_alt, count,
                                status, cap, ranges, order, image, T_final, last_idx)
            inst = state.instances()
            _lib.check("gs_bin", lib.gs_bin(ctypes.byref(proj), n, cams_c, V, cfg,
                                            ctypes.byref(inst), _lib.ptr(bin_ws),
                                            bin_ws.numel(), stream))
            sort_bytes = lib.gs_sort_workspace_bytes(cap, n_tiles, cfg)
            sort_ws = torch.empty(max(1, sort_bytes), dtype=torch.uint8, device=dev)
            _lib.check("gs_sort", lib.gs_sort(ctypes.byref(inst), n_tiles, cfg,
                                              _lib.ptr(ranges), _lib.ptr(order), _lib.ptr(sort_ws),
                                              sort_ws.numel(), stream))
            _lib.check("gs_render_fwd", lib.gs_render_fwd(
                ctypes.byref(proj), ctypes.byref(inst), _lib.ptr(ranges), _lib.ptr(order), cams_c,
                V, cfg, _lib.ptr(image), _lib.ptr(T_final) if for_backward else 0,
                _lib.ptr(last_idx) if for_backward else 0, n, stream))
            if not check:
                break
            st, ct = state.read_status()
            if st & _lib.STATUS_CAPACITY:
                if ct > _lib.MAX_INSTANCES:
                    raise _lib.GsError("gs_bin", _lib.ERR_UNSUPPORTED)
                cap = max(int(ct * self.growth) + 1, cap + 1)
                continue
            if st & _lib.STATUS_SORT:
                raise _lib.GsError("gs_sort", _lib.ERR_SORT)
            break
        self.capacity = cap
        return state

    # -- backward ----------------------------------------------------------------
    def backward(self, params: GaussianParams, state: RenderState,
                 dL_dimage: torch.Tensor | None = None, l1=None):
        """Gradients of the raw parameters (dict of tensors shaped like ``params``), from
        an upstream dL/dimage, or with ``l1=(target, loss)`` for the L1 loss alone taken
        inside the backward blend (gs_render_bwd_l1): the per-view losses are added to
        ``loss`` (a [V] tensor, or None), as l1_loss_grad does."""
        lib = _lib.lib()
        dev = params.means.device
        stream = torch.cuda.current_stream(dev).cuda_stream
        cfg = ctypes.byref(self.cfg)
        V, n = state.n_views, state.n
        if state.T_final.numel() == 0:
            raise ValueError("the state was rendered with for_backward=False")
        if (dL_dimage is None) == (l1 is None):
            raise ValueError("give either dL_dimage or l1=(target, loss)")
        grad2d = torch.zeros(max(1, V * n * _lib.GRAD2D_FLOATS), dtype=torch.float32, device=dev)
        proj = state.projected()
        inst = state.instances()
        if l1 is None:
            if dL_dimage.numel() != state.image.numel() or dL_dimage.dtype != torch.float32:
                raise ValueError("dL_dimage must match the flat float32 image layout")
            dL_dimage = dL_dimage.contiguous()
            _lib.check("gs_render_bwd", lib.gs_render_bwd(
                ctypes.byref(proj), ctypes.byref(inst), _lib.ptr(state.ranges), _lib.ptr(state.order),
                state.cams_c, V, cfg,
                _lib.ptr(state.T_final), _lib.ptr(state.last_idx), _lib.ptr(dL_dimage),
                _lib.ptr(grad2d), n, stream))
        else:
            target, loss = l1
            if target.numel() != state.image.numel() or target.dtype != torch.float32:
                raise ValueError("the L1 target must match the flat float32 image layout")
            target = target.contiguous()
            ws = torch.empty(max(1, lib.gs_render_l1_workspace_bytes(state.cams_c, V, cfg)),
                             dtype=torch.uint8, device=dev)
            _lib.check("gs_render_bwd_l1", lib.gs_render_bwd_l1(
                ctypes.byref(proj), ctypes.byref(inst), _lib.ptr(state.ranges), _lib.ptr(state.order),
                state.cams_c, V, cfg, _lib.ptr(state.T_final), _lib.ptr(state.last_idx),
                _lib.ptr(state.image), _lib.ptr(target), _lib.ptr(grad2d), _lib.ptr(loss),
                _lib.ptr(ws), ws.numel(), n, stream))
        grads = {k: torch.empty_like(getattr(params, k))
                 for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
        k_active = (self.cfg.sh_degree + 1) ** 2
        if grads["sh"].shape[0] > k_active:
            grads["sh"][k_active:].zero_()      # bands not yet active get no gradient
        gp = _lib.GsParamsGrad(*(_lib.ptr(grads[k]) for k in
                                 ("means", "log_scales", "quats", "opacity_logits", "sh")))
        pr = params.c_struct()
        _lib.check("gs_project_bwd", lib.gs_project_bwd(
            ctypes.byref(pr), state.cams_c, V, cfg, ctypes.byref(proj), _lib.ptr(grad2d),
            ctypes.byref(gp), stream))
        return grads, grad2d


class RasterizeFunction(torch.autograd.Function):
    """Differentiable rasterization: returns the flat image of all views (see RenderState)."""

    @staticmethod
    def forward(ctx, rasterizer, cams, means, log_scales, quats, opacity_logits, sh):
        params = GaussianParams(means.contiguous(), log_scales.contiguous(), quats.contiguous(),
                                opacity_logits.contiguous(), sh.contiguous())
        state = rasterizer.render(params, cams, check=rasterizer.check)
        ctx.rasterizer = rasterizer
        ctx.state = state
        ctx.params = params
        return state.image

    @staticmethod
    def backward(ctx, dL_dimage):
        grads, _ = ctx.rasterizer.backward(ctx.params, ctx.state, dL_dimage.float())
        return (None, None, grads["means"], grads["log_scales"], grads["quats"],
                grads["opacity_logits"], grads["sh"])


def l1_loss_grad(state: RenderState, target: torch.Tensor, loss: torch.Tensor | None = None):
    """dL/dimage of the per-view mean L1 loss (flat image layout); adds the losses to ``loss``."""
    dL = torch.empty_like(state.image)
    stream = torch.cuda.current_stream(state.image.device).cuda_stream
    _lib.check("gs_loss_l1", _lib.lib().gs_loss_l1(
        _lib.ptr(state.image), _lib.ptr(target), state.cams_c, state.n_views, _lib.ptr(dL),
        _lib.ptr(loss), stream))
    return dL


def photometric_loss_grad(state: RenderState, target: torch.Tensor, lam: float = 0.2,
                          loss: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """dL/dimage of (1 - lam) L1 + lam D-SSIM per view (Sec. 5.1); adds the losses to ``loss``."""
    lib = _lib.lib()
    dL = torch.empty_like(state.image)
    need = lib.gs_loss_workspace_bytes(state.cams_c, state.n_views)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=state.image.device)
    stream = torch.cuda.current_stream(state.image.device).cuda_stream
    _lib.check("gs_loss_photometric", lib.gs_loss_photometric(
        _lib.ptr(state.image), _lib.ptr(target), state.cams_c, state.n_views, float(lam),
        _lib.ptr(dL), _lib.ptr(loss), _lib.ptr(workspace), workspace.numel(), stream))
    return dL


def rasterize(rasterizer: Rasterizer, cams, means, log_scales, quats, opacity_logits, sh):
    """Autograd entry point: flat image (per view [3][H][W], concatenated)."""
    return RasterizeFunction.apply(rasterizer, list(cams), means, log_scales, quats,
                                   opacity_logits, sh)


class GraphStep:
    """One step (forward, backward with the L1 loss taken inside it) captured in a HIP graph.

    Every call of the captured sequence only enqueues kernels and allocates nothing
    outside torch's graph pool, so a replay re-runs the whole hot path with one
    launch. Parameters and targets are read from the tensors given here: update
    them in place between replays. After a replay, ``outputs.state.read_status()``
    (which synchronises) reports an instance-capacity overflow; then build a new
    GraphStep with a larger ``rasterizer.capacity``.
    """

    def __init__(self, rasterizer: Rasterizer, params: GaussianParams, cams, target: torch.Tensor,
                 warmup: int = 2):
        if rasterizer.capacity is None:
            raise ValueError("set rasterizer.capacity (e.g. from one checked render) before capture")
        self.rast = rasterizer
        self.params = params
        self.cams = list(cams)
        self.target = target
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self._body()
        torch.cuda.current_stream().wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.state, self.grads, self.loss = self._body()

    def _body(self):
        state = self.rast.render(self.params, self.cams, check=False)
        loss = torch.zeros(len(self.cams), dtype=torch.float32, device=state.image.device)
        grads, _ = self.rast.backward(self.params, state, l1=(self.target, loss))
        return state, grads, loss

    def replay(self):
        self.graph.replay()
        return self.state, self.grads, self.loss
