"""Benchmark: 1080p forward+backward views/s at 3M Gaussians, batched vs per-view.

One step = the whole hot path over one batch of views: project -> bin -> sort ->
blend forward -> L1 loss gradient -> blend backward -> projection backward, on
seeded synthetic inputs resident in HBM (default: 3M Gaussians of the clustered-scene
generator, SH degree 3, four 1920x1080 orbit cameras; targets rendered once from a
jittered copy of the scene). ``value`` is the batched rate: all views of a step in one
call per stage, the step captured as one HIP graph. Beside it: the same batched step
launched eagerly, and the step done one view at a time (eager, and one graph per view).

Prints one JSON line (rank 0). Runs on one GPU: --gpus above 1 exits with a message.
``--mode train`` runs the Adam training loop instead (steps/s and peak HBM).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak in lane operations per second (an FMA counted once): the published
# 157.3 TFLOP/s (an FMA counted as two flops) = 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz.
# The kernels reach VALU issue rates above the 16-lanes-per-SIMD figure, so the
# 32-lane figure is the ceiling that applies.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12


WORKLOAD_TEXT = {
    "train4": "clustered scene, {n} Gaussians, SH3, {v} orbit views of 1920x1080 per step, "
              "fwd+bwd with L1 loss, batched: all views in one call per stage, one HIP graph "
              "per step",
    "full1080": "clustered scene, {n} Gaussians, SH3, one 1920x1080 view at the origin, "
                "fwd+bwd with L1 loss, one HIP graph per step",
    "multiview": "clustered scene, {n} Gaussians, SH3, {v} orbit views of mixed resolution "
                 "(640x360 to 1920x1080), fwd+bwd with L1 loss, batched, one HIP graph per step",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--views", type=int, default=4)
    ap.add_argument("--n", type=int, default=None, help="Gaussians (default: the workload's)")
    ap.add_argument("--workload", choices=("train4", "full1080", "multiview"), default="train4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--mode", choices=("views", "train"), default="views",
                    help="views: the fwd+bwd views/s metric (default); train: the Adam training "
                         "loop over 4-view minibatches (steps/s and peak HBM)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (the reference kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    if args.mode == "train":
        return train(args)
    import numpy as np
    import torch

    import scenes
    from paper_2308_04079_amd import GaussianParams, Rasterizer
    from paper_2308_04079_amd.raster import GraphStep, l1_loss_grad

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731

    t0 = time.time()
    sc, cams = scenes.workload(args.workload, args.n)
    if args.workload == "train4" and args.views != 4:
        cams = scenes.orbit_cameras(args.views, 4, resolutions=((1920, 1080),))
    target_sc = scenes.jitter_means(sc, 4)
    params = GaussianParams.from_numpy(sc, dev)
    tparams = GaussianParams.from_numpy(target_sc, dev)
    del target_sc
    V = len(cams)
    log(f"[bench] scene ready in {time.time() - t0:.1f}s: N={sc.n}, {V} views")

    rast = Rasterizer(sh_degree=sc.sh_degree)
    tstate = rast.render(tparams, cams)             # sizes the capacity and renders targets
    target = tstate.image.clone()
    del tstate, tparams
    probe = rast.render(params, cams)
    st, count = probe.read_status()
    rast.capacity = int(count * 1.15) + 4096
    del probe
    zero_loss = torch.zeros(V, dtype=torch.float32, device=dev)

    def step(rs, cam_list, tgt):
        state = rs.render(params, cam_list, check=False)
        loss = zero_loss[:len(cam_list)].clone()
        dL = l1_loss_grad(state, tgt, loss)
        grads, _ = rs.backward(params, state, dL)
        return state, grads, loss

    def timed(fn, steps, dist=None):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if dist is not None else []
        torch.cuda.synchronize()
        a = time.perf_counter()
        for k in range(steps):
            if evs:
                evs[k].record()
            out = fn()
        if evs:
            evs[steps].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - a
        if evs:
            dist.extend(evs[k].elapsed_time(evs[k + 1]) for k in range(steps))
        return out, wall

    # headline: the whole batched step as one HIP graph launch
    gstep = GraphStep(rast, params, cams, target, warmup=max(args.warmup, 1))
    for _ in range(args.warmup):
        gstep.replay()
    step_ms = []
    (state, grads, loss), dt = timed(gstep.replay, args.steps, step_ms)
    st, count = state.read_status()
    assert st == 0, f"device status {st} in the timed region"
    ms_per_step = dt * 1000.0 / args.steps
    views_per_s = V * args.steps / dt
    log(f"[bench] batched, one graph per step: {ms_per_step:.2f} ms/step, {views_per_s:.1f} views/s"
        f" (M={count} instances)")

    # the same batched step launched eagerly, call by call
    for _ in range(args.warmup):
        step(rast, cams, target)
    _, dt_e = timed(lambda: step(rast, cams, target), args.steps)
    eager_views = V * args.steps / dt_e
    log(f"[bench] batched, eager launches: {eager_views:.1f} views/s")

    # kernel-level timing of every library call, with events on the launch stream
    stages = time_stages(rast, params, cams, target, args.steps, zero_loss)
    log("[bench] stages (ms): " + ", ".join(f"{k}={v:.3f}" for k, v in stages["ms"].items()))

    per_view = per_view_graph = None
    if not args.no_per_view:
        prast = Rasterizer(sh_degree=sc.sh_degree, capacity=rast.capacity)
        tviews = [target[3 * state.pix_offset[v]:3 * state.pix_offset[v + 1]] for v in range(V)]

        def per_view_step():
            for v in range(V):
                step(prast, [cams[v]], tviews[v])
        for _ in range(args.warmup):
            per_view_step()
        _, dt_p = timed(per_view_step, args.steps)
        per_view = V * args.steps / dt_p
        graphs = [GraphStep(prast, params, [cams[v]], tviews[v]) for v in range(V)]

        def per_view_graph_step():
            for g in graphs:
                g.replay()
        for _ in range(args.warmup):
            per_view_graph_step()
        _, dt_pg = timed(per_view_graph_step, args.steps)
        per_view_graph = V * args.steps / dt_pg
        del graphs
        log(f"[bench] per-view: {per_view:.1f} views/s eager, {per_view_graph:.1f} views/s graphs")

    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy probe: 268435456 bytes read, 268435456 bytes written")
        del src, dst

    roof = roofline(stages, state, count, sc.n, V, rast.cfg)
    hbm = hbm_rates(stages["ms"], stages["state"], count, sc.n, V, (sc.sh_degree + 1) ** 2,
                    rast.cfg.sort_digit_bits)
    q = np.percentile(np.array(step_ms), [10, 50, 90])
    cpu = None if args.no_cpu_baseline else cpu_baseline(log)

    out = {
        "metric": "1080p fwd+bwd views/sec at 3M Gaussians, batched vs per-view, <=1e-4 image err",
        "value": round(views_per_s, 3),
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload].format(n=sc.n, v=V),
                   "gaussians": sc.n, "views_per_step": V,
                   "resolutions": sorted({f"{c.width}x{c.height}" for c in cams}),
                   "tile": 16, "sort_digit_bits": 8, "lds_batch": 64, "instances": count},
        "batched_eager_value": round(eager_views, 3),
        "per_view_value": None if per_view is None else round(per_view, 3),
        "per_view_graph_value": None if per_view_graph is None else round(per_view_graph, 3),
        "step_ms_p10_p50_p90": [round(float(x), 4) for x in q],
        "stage_ms": {k: round(v, 4) for k, v in stages["ms"].items()},
        "stage_hbm": hbm,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def train(args):
    """The optimisation loop of Alg. 1 on the library: 3M Gaussians, SH3, 4 distinct
    1920x1080 views per step drawn (seeded) from a pool of 64 orbit cameras, the
    L1 + 0.2 D-SSIM loss against targets rendered once from a jittered copy of the
    scene, Adam on every parameter group, density statistics accumulated every step.
    Warm-up resolution and the SH ramp are off (full resolution, all bands) and no
    densification falls inside the timed steps, so every step does the same work."""
    import numpy as np
    import torch

    import scenes
    from paper_2308_04079_amd import GaussianParams, Rasterizer
    from paper_2308_04079_amd.train import TrainConfig, Trainer

    dev = torch.device("cuda:0")
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    sc = scenes.clustered_scene(args.n or 3_000_000, 4, 3)
    pool = scenes.orbit_cameras(64, 40, resolutions=((1920, 1080),))
    tparams = GaussianParams.from_numpy(scenes.jitter_means(sc, 4), dev)
    rast = Rasterizer(sh_degree=3)
    targets = [rast.render(tparams, [cam]).image.clone() for cam in pool]
    del tparams
    total = args.warmup + args.steps
    cfg = TrainConfig(iterations=total, views_per_step=4, warmup=(0, 0), sh_every=0,
                      densify_from=total + 1, densify_until=total, reset_every=10 ** 9)
    tr = Trainer(GaussianParams.from_numpy(sc, dev), pool, targets, extent=20.0, cfg=cfg)
    for _ in range(args.warmup):
        tr.step()
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats(dev)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tr.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    losses = [float(x.sum()) for x in tr.history[args.warmup:]]
    log(f"[train] {args.steps} steps in {dt:.2f}s, loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    print(json.dumps({
        "metric": "training steps/sec (3M Gaussians, 4x1920x1080 views per step, fwd+bwd+Adam)",
        "value": round(args.steps / dt, 3), "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1000 / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"clustered scene, {sc.n} Gaussians, SH3, Adam over 4 of 64 "
                               "orbit 1920x1080 views per step, L1 + 0.2 D-SSIM loss, "
                               "density statistics",
                   "gaussians": sc.n, "views_per_step": 4},
        "peak_hbm_bytes": int(torch.cuda.max_memory_allocated(dev)),
        "loss_first": losses[0], "loss_last": losses[-1]}), flush=True)


def time_stages(rast, params, cams, target, steps, zero_loss):
    """Average duration of each library call over `steps` steps, HIP events on the stream."""
    import ctypes

    import torch

    from paper_2308_04079_amd import _lib
    lib = _lib.lib()
    names = ["project", "bin", "sort", "render_fwd", "loss", "render_bwd", "project_bwd"]
    acc = {k: 0.0 for k in names}
    for _ in range(steps):
        st = rast.render(params, cams, check=False)
        # re-issue each stage on the same buffers, bracketed by events
        stream = torch.cuda.current_stream().cuda_stream
        cfg = ctypes.byref(rast.cfg)
        proj, inst = st.projected(), st.instances()
        pr = params.c_struct()
        V, n = st.n_views, st.n
        bin_ws = torch.empty(max(1, lib.gs_bin_workspace_bytes(V * n, cfg)), dtype=torch.uint8,
                             device="cuda")
        sort_ws = torch.empty(max(1, lib.gs_sort_workspace_bytes(st.capacity, st.n_tiles, cfg)),
                              dtype=torch.uint8, device="cuda")
        dL = torch.empty_like(st.image)
        loss = zero_loss[:V].clone()
        grad2d = torch.zeros(V * n * _lib.GRAD2D_FLOATS, dtype=torch.float32, device="cuda")
        grads = {k: torch.empty_like(getattr(params, k))
                 for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
        gp = _lib.GsParamsGrad(*(_lib.ptr(grads[k]) for k in
                                 ("means", "log_scales", "quats", "opacity_logits", "sh")))
        calls = [
            ("project", lambda: lib.gs_project(ctypes.byref(pr), st.cams_c, V, cfg,
                                               ctypes.byref(proj), stream)),
            ("bin", lambda: lib.gs_bin(ctypes.byref(proj), n, st.cams_c, V, cfg,
                                       ctypes.byref(inst), _lib.ptr(bin_ws), bin_ws.numel(),
                                       stream)),
            ("sort", lambda: lib.gs_sort(ctypes.byref(inst), st.n_tiles, cfg, _lib.ptr(st.ranges),
                                         _lib.ptr(st.order), _lib.ptr(sort_ws), sort_ws.numel(),
                                         stream)),
            ("render_fwd", lambda: lib.gs_render_fwd(
                ctypes.byref(proj), ctypes.byref(inst), _lib.ptr(st.ranges), _lib.ptr(st.order),
                st.cams_c, V, cfg, _lib.ptr(st.image), _lib.ptr(st.T_final), _lib.ptr(st.last_idx), n, stream)),
            ("loss", lambda: lib.gs_loss_l1(_lib.ptr(st.image), _lib.ptr(target), st.cams_c, V,
                                            _lib.ptr(dL), _lib.ptr(loss), stream)),
            ("render_bwd", lambda: lib.gs_render_bwd(
                ctypes.byref(proj), ctypes.byref(inst), _lib.ptr(st.ranges), _lib.ptr(st.order),
                st.cams_c, V, cfg, _lib.ptr(st.T_final), _lib.ptr(st.last_idx), _lib.ptr(dL), _lib.ptr(grad2d), n,
                stream)),
            ("project_bwd", lambda: lib.gs_project_bwd(ctypes.byref(pr), st.cams_c, V, cfg,
                                                       ctypes.byref(proj), _lib.ptr(grad2d),
                                                       ctypes.byref(gp), stream)),
        ]
        evs = []
        for name, fn in calls:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            rc = fn()
            b.record()
            assert rc == 0, (name, rc)
            evs.append((name, a, b))
        torch.cuda.synchronize()
        for name, a, b in evs:
            acc[name] += a.elapsed_time(b)
    st_last = st
    return {"ms": {k: v / steps for k, v in acc.items()}, "state": st_last}


def kernel_source_hash():
    import hashlib
    path = os.path.join(ROOT, "paper_2308_04079_amd", "csrc", "gs_render.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    or None when the kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "render_traffic_full1080x4.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256_16") != kernel_source_hash() or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel]["hbm_bytes_per_launch"]


def processed_pairs(st, cfg, T=16):
    """(wave, Gaussian) pairs the blend-backward launch evaluates.

    A wave owns an 8x8 pixel block of a tile; it walks the tile's list from the
    block's last contributor back to the start and evaluates (on all 64 lanes)
    every entry whose 3-sigma pixel box meets its block and whose least Mahalanobis
    distance m over the block's pixel-centre rectangle is within
    min(9, 2 ln(o / alpha_min)) (the kernel's two staging tests, replayed here in
    FP64 without the kernel's rounding slack).
    """
    import torch
    dev = st.ranges.device
    M = int(st.count.item())
    vals = st.vals[:M].long() & 0xFFFFFFFF
    tile = st.tile_ids(cfg)[:M].long()
    rec = st.record.view(-1, 12)
    lo = rec[vals, 0].view(torch.int32).long()
    hi = rec[vals, 1].view(torch.int32).long()
    ilo, jlo, ihi, jhi = lo & 0xFFFF, (lo >> 16) & 0xFFFF, hi & 0xFFFF, (hi >> 16) & 0xFFFF
    mx, my = rec[vals, 2].double(), rec[vals, 3].double()
    w00, w10, w11 = rec[vals, 4].double(), rec[vals, 5].double(), rec[vals, 6].double()
    opac = rec[vals, 7].double()
    thr_all = torch.clamp(2.0 * (torch.log(opac) - math.log(cfg.alpha_min)), max=cfg.sigma_extent ** 2)
    pos = torch.arange(M, device=dev)
    toff = torch.tensor(st.tile_offset, device=dev)
    view = torch.searchsorted(toff, tile, right=True) - 1
    total = 0
    for v in range(st.n_views):
        cam = st.cams[v]
        W, H = cam.width, cam.height
        tx_n, ty_n = (W + T - 1) // T, (H + T - 1) // T
        last = st.view_plane(st.last_idx, v).long()
        # per 8x8 block: the largest last index (-1 if none)
        Hp, Wp = ty_n * T, tx_n * T
        pad = torch.full((Hp, Wp), -1, dtype=torch.long, device=dev)
        pad[:H, :W] = last
        blk = pad.view(Hp // 8, 8, Wp // 8, 8).amax(dim=(1, 3))          # (Hp/8, Wp/8)
        sel = view == v
        t_local = tile[sel] - st.tile_offset[v]
        tyi, txi = t_local // tx_n, t_local % tx_n
        for qy in range(T // 8):
            for qx in range(T // 8):
                by, bx = tyi * (T // 8) + qy, txi * (T // 8) + qx
                x0, y0 = bx * 8, by * 8
                inside = (x0 < W) & (y0 < H)
                x1, y1 = torch.clamp(x0 + 7, max=W - 1), torch.clamp(y0 + 7, max=H - 1)
                ov = (ilo[sel] <= x1) & (ihi[sel] >= x0) & (jlo[sel] <= y1) & (jhi[sel] >= y0)
                dxa = (x0 - ilo[sel]) + 0.5 - mx[sel]
                dxb = (x1 - ilo[sel]) + 0.5 - mx[sel]
                dya = (y0 - jlo[sel]) + 0.5 - my[sel]
                dyb = (y1 - jlo[sel]) + 0.5 - my[sel]
                a00, a10, a11 = w00[sel], w10[sel], w11[sel]

                def edge_x(X):   # least m on the edge dx = X: vertex of the parabola, clamped
                    dy = torch.minimum(torch.maximum(-a10 * X / a11, dya), dyb)
                    return (a00 * X) ** 2 + (a10 * X + a11 * dy) ** 2

                def edge_y(Y):
                    dx = torch.minimum(torch.maximum(-a10 * a11 * Y / (a00 ** 2 + a10 ** 2), dxa), dxb)
                    return (a00 * dx) ** 2 + (a10 * dx + a11 * Y) ** 2

                mmin = torch.minimum(torch.minimum(edge_x(dxa), edge_x(dxb)),
                                     torch.minimum(edge_y(dya), edge_y(dyb)))
                inside_rect = (dxa <= 0) & (dxb >= 0) & (dya <= 0) & (dyb >= 0)
                mmin = torch.where(inside_rect, torch.zeros_like(mmin), mmin)
                ov &= mmin <= thr_all[sel]
                wl = blk[by.clamp(max=blk.shape[0] - 1), bx.clamp(max=blk.shape[1] - 1)]
                total += int((inside & ov & (pos[sel] <= wl)).sum().item())
    return total


def roofline(stages, state, count, n, V, cfg):
    """Roofline of the dominant kernel. For the blend kernels (VALU bound): lane
    evaluations actually issued (processed pairs x 64) x the arithmetic of one
    evaluation (FWD_OPS_PER_EVAL, BWD_OPS_PER_EVAL), against the FP32 VALU peak."""
    ms = stages["ms"]
    dom = max(("render_fwd", "render_bwd", "project", "project_bwd", "sort"), key=lambda k: ms[k])
    st = stages["state"]
    if dom in ("render_bwd", "render_fwd"):
        pairs = processed_pairs(st, cfg)
        ops = BWD_OPS_PER_EVAL if dom == "render_bwd" else FWD_OPS_PER_EVAL
        lane_evals = pairs * 64
        achieved = lane_evals * ops / (ms[dom] * 1e-3) / 1e12
        return {"kernel": dom, "bound": "alu", "achieved": round(achieved, 3),
                "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s (FP32 VALU lane-ops)",
                "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": measured_traffic(dom),
                "units": {"wave_gaussian_pairs": pairs, "lane_evaluations": lane_evals,
                          "ops_per_evaluation": ops}}
    K = 16
    per = {"project": (4 * (11 + 3 * K) + 56 * V), "project_bwd": (4 * (11 + 3 * K) * 2 + 40 * V)}
    b = per.get(dom, 24) * (n if dom in per else count)
    achieved = b / (ms[dom] * 1e-3) / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}


def hbm_rates(ms, st, count, n, V, K, digit_bits):
    """Algorithmic HBM bytes of the streaming stages and the rate each reaches.

    project: parameters once (4 (11 + 3K) B per Gaussian) + depth key and tile count
    per (view, Gaussian) + a 48 B record per visible one; bin: tile counts read once,
    per visible pair its depth key and pixel box read, 16 B moved per depth-sort pass
    (key and value read and written), 8 B written per instance; sort: 16 B per
    instance per tile-id pass; project_bwd: parameters read and gradients written
    (2 x 4 (11 + 3K) B per Gaussian), tile counts, and per visible (view, Gaussian) its
    record and its 36 B screen-space gradient.
    """
    from paper_2308_04079_amd import _lib
    vis = int((st.tiles_touched[:V * n] > 0).sum().item())
    par = 4 * (11 + 3 * K)
    tile_passes = -(-_lib.lib().gs_sort_key_bits(st.n_tiles) // digit_bits)
    depth_passes = -(-31 // digit_bits)
    b = {"project": par * n + 8 * V * n + 48 * vis,
         "bin": 4 * V * n + (12 + 16 * depth_passes) * vis + 8 * count,
         "sort": 16 * count * tile_passes,
         "project_bwd": 2 * par * n + 4 * V * n + (48 + 36) * vis}
    out = {}
    for k, v in b.items():
        gbs = v / (ms[k] * 1e-3) / 1e9
        out[k] = {"bytes": v, "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["bin"]["depth_passes"] = depth_passes
    out["sort"]["passes"] = tile_passes
    out["visible_pairs"] = vis
    return out


# FP32 VALU operations of one (pixel, Gaussian) evaluation as the method states it
# (one op per add, mul, fma, compare, select, min, exp, reciprocal). Forward, 22:
# offset 4, Mahalanobis 5, exp argument and exp 2, alpha 2, three tests 3, T' 2,
# weight and colour accumulation 4. Backward, 57: the forward's 16 evaluation ops,
# T recovery 3, colour gradient 4, alpha gradient 10, back-to-front accumulator 3,
# clamp test 2, opacity / mean / whitening gradients 10, and the 9 adds that sum the
# pixel's nine partial gradients into the Gaussian's totals (the accumulation the
# forward's count includes for the colour).
FWD_OPS_PER_EVAL = 22
BWD_OPS_PER_EVAL = 57


def cpu_baseline(log):
    """The FP64 oracle timed on a bounded sample of one view of the same workload, with
    NumPy's thread pools held to one thread (``cores`` = 1)."""
    from threadpoolctl import threadpool_limits

    import scenes
    from oracle.rules import Rules

    sc = scenes.clustered_scene(3_000_000, 4, 3)
    cam = scenes.orbit_cameras(1, 4, resolutions=((1920, 1080),))[0]
    r = Rules()
    with threadpool_limits(limits=1):       # BLAS and OpenMP pools: one thread
        return _cpu_baseline_timed(sc, cam, r, log)


def _cpu_baseline_timed(sc, cam, r, log):
    import numpy as np

    from oracle.adjoint import blend_backward, empty_acc, project_backward
    from oracle.gaussians import project
    from oracle.raster import tile_lists, tile_pixels
    t = time.perf_counter()
    p = project(sc, cam, r)
    t_proj = time.perf_counter() - t
    t = time.perf_counter()
    tl = tile_lists(p, r)
    t_lists = time.perf_counter() - t
    n_tiles = tl.tiles_x * tl.tiles_y
    rng = np.random.default_rng(0)
    sample = rng.choice(n_tiles, 16, replace=False)
    acc = empty_acc(p.n)
    w = rng.standard_normal((cam.height, cam.width, 3))
    t = time.perf_counter()
    for tt in sample:
        px, py = tile_pixels(int(tt), tl, cam.width, cam.height, r.tile)
        ids = tl.ids[tl.start[tt]:tl.start[tt + 1]]
        blend_backward(p, ids, px, py, w[py, px], r, acc)
    t_tiles = time.perf_counter() - t
    t = time.perf_counter()
    project_backward(sc, p, acc)
    t_pbwd = time.perf_counter() - t
    per_view_s = t_proj + t_lists + t_tiles * n_tiles / len(sample) + t_pbwd
    log(f"[bench] oracle: project {t_proj:.1f}s lists {t_lists:.1f}s "
        f"{len(sample)} tiles fwd+bwd {t_tiles:.1f}s project_bwd {t_pbwd:.1f}s "
        f"-> {per_view_s:.0f}s per view")
    return {"value": round(1.0 / per_view_s, 6), "unit": "views/s", "cores": 1, "kind": "oracle",
            "sample": f"one 1920x1080 view of the 3M-Gaussian workload: full projection, tile "
                      f"lists and projection backward, fwd+bwd blend of {len(sample)} of "
                      f"{n_tiles} tiles scaled to the whole frame; single-threaded NumPy FP64"}


if __name__ == "__main__":
    main()
