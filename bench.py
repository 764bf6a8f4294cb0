"""Benchmark: 1080p forward+backward views/s at 3M Gaussians, batched vs per-view.

One step = the whole hot path over one batch of views: project -> bin -> sort ->
blend forward -> blend backward with the L1 loss and its gradient formed inside it ->
projection backward, on
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
    ap.add_argument("--mode", choices=("views", "train", "oracle"), default="views",
                    help="views: the fwd+bwd views/s metric (default); train: the Adam training "
                         "loop over 4-view minibatches (steps/s and peak HBM); oracle: the CPU "
                         "oracle's seconds per view on the parity workloads (no GPU)")
    ap.add_argument("--tile", type=int, default=None, help="tile size (default: autotuned)")
    ap.add_argument("--lds-batch", type=int, default=None,
                    help="list entries staged per wave and round (default: autotuned)")
    ap.add_argument("--digit-bits", type=int, default=None,
                    help="radix digit width of the sorts (default: autotuned)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (the reference kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; runs over several GPUs are not part of it (use --gpus 1)"}))
        sys.exit(2)
    if args.mode == "train":
        return train(args)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    if args.mode == "oracle":
        return oracle_table(log)
    # the oracle runs first, in worker processes forked before this process touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(log)
    import numpy as np
    import torch

    import scenes
    from paper_2308_04079_amd import GaussianParams, Rasterizer
    from paper_2308_04079_amd.raster import GraphStep

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

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

    knobs = {k: v for k, v in (("tile_size", args.tile), ("lds_batch", args.lds_batch),
                               ("sort_digit_bits", args.digit_bits)) if v is not None}
    tstate = Rasterizer(sh_degree=sc.sh_degree, **knobs).render(tparams, cams)
    target = tstate.image.clone()                   # the targets do not depend on the knobs
    del tstate, tparams
    tuned = None
    if len(knobs) < 3:
        # the autotuner times one fwd + L1 + bwd step per combination of the knobs not
        # given on the command line, on this workload
        from paper_2308_04079_amd.autotune import DIGIT_BITS, LDS_BATCHES, TILE_SIZES, autotune
        t0 = time.time()
        tuned = autotune(params, cams, target, steps=2, use_cache=False,
                         tile_sizes=(knobs["tile_size"],) if "tile_size" in knobs else TILE_SIZES,
                         lds_batches=(knobs["lds_batch"],) if "lds_batch" in knobs else LDS_BATCHES,
                         digit_bits=(knobs["sort_digit_bits"],) if "sort_digit_bits" in knobs
                         else DIGIT_BITS)
        knobs = {k: tuned[k] for k in ("tile_size", "lds_batch", "sort_digit_bits")}
        log(f"[bench] autotune ({len(tuned['trials'])} trials, {time.time() - t0:.0f}s): {knobs}")
    rast = Rasterizer(sh_degree=sc.sh_degree, **knobs)
    probe = rast.render(params, cams)
    st, count = probe.read_status()
    rast.capacity = int(count * 1.15) + 4096
    del probe
    zero_loss = torch.zeros(V, dtype=torch.float32, device=dev)

    def step(rs, cam_list, tgt):
        state = rs.render(params, cam_list, check=False)
        loss = zero_loss[:len(cam_list)].clone()
        # the L1 gradient is formed inside the backward blend (gs_render_bwd_l1)
        grads, _ = rs.backward(params, state, l1=(tgt, loss))
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
        prast = Rasterizer(sh_degree=sc.sh_degree, capacity=rast.capacity, **knobs)
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
                   "tile": rast.cfg.tile_size, "sort_digit_bits": rast.cfg.sort_digit_bits,
                   "lds_batch": rast.cfg.lds_batch, "instances": count},
        "batched_eager_value": round(eager_views, 3),
        "per_view_value": None if per_view is None else round(per_view, 3),
        "per_view_graph_value": None if per_view_graph is None else round(per_view_graph, 3),
        "step_ms_p10_p50_p90": [round(float(x), 4) for x in q],
        "stage_ms": {k: round(v, 4) for k, v in stages["ms"].items()},
        "stage_hbm": hbm,
        "roofline": roof,
        "cpu_baseline": cpu,
        "autotune": None if tuned is None else {
            "chosen": knobs, "trials": [{k: (round(v, 4) if k == "ms" else v) for k, v in t.items()}
                                        for t in tuned["trials"]]},
    }
    print(json.dumps(out), flush=True)


def train(args):
    """The optimisation loop of Alg. 1 on the library: 3M Gaussians, SH3, 4 distinct
    1920x1080 views per step drawn (seeded) from a pool of 64 orbit cameras, the
    L1 + 0.2 D-SSIM loss against targets rendered once from a jittered copy of the
    scene, Adam on every parameter group, density statistics accumulated every step and
    density control (clone, split, prune) every 100 iterations, inside the timed steps.
    Warm-up resolution and the SH ramp are off (full resolution, all bands); no opacity
    reset falls within 200 steps (its cadence is 3000)."""
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
                      densify_from=1, densify_until=total)
    tr = Trainer(GaussianParams.from_numpy(sc, dev), pool, targets, extent=20.0, cfg=cfg)
    for _ in range(args.warmup):
        tr.step()
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats(dev)
    n_start = tr.params.n
    t0 = time.perf_counter()
    for k in range(args.steps):
        tr.step()
        if (k + 1) % 50 == 0:
            log(f"[train] step {k + 1}: {tr.params.n} Gaussians")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_densify = sum(1 for it in range(args.warmup + 1, total + 1) if tr.densify_now(it))
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
                               "density statistics every step and density control every "
                               "100 iterations",
                   "gaussians": sc.n, "views_per_step": 4},
        "gaussians_timed_start": n_start, "gaussians_timed_end": tr.params.n,
        "densifications_timed": n_densify,
        "peak_hbm_bytes": int(torch.cuda.max_memory_allocated(dev)),
        "loss_first": losses[0], "loss_last": losses[-1]}), flush=True)


def time_stages(rast, params, cams, target, steps, zero_loss):
    """Average duration of each library call over `steps` steps, HIP events on the stream."""
    import ctypes

    import torch

    from paper_2308_04079_amd import _lib
    lib = _lib.lib()
    names = ["project", "bin", "sort", "render_fwd", "render_bwd", "project_bwd"]
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
        loss = zero_loss[:V].clone()
        l1_ws = torch.empty(max(1, lib.gs_render_l1_workspace_bytes(st.cams_c, V, cfg)),
                            dtype=torch.uint8, device="cuda")
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
            ("render_bwd", lambda: lib.gs_render_bwd_l1(
                ctypes.byref(proj), ctypes.byref(inst), _lib.ptr(st.ranges), _lib.ptr(st.order),
                st.cams_c, V, cfg, _lib.ptr(st.T_final), _lib.ptr(st.last_idx), _lib.ptr(st.image),
                _lib.ptr(target), _lib.ptr(grad2d), _lib.ptr(loss), _lib.ptr(l1_ws), l1_ws.numel(),
                n, stream)),
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


def backward_work(st, cfg):
    """Work units of one gs_render_bwd launch, counted from the sorted instances and the
    forward state outside the timed region.

    The kernel runs one 64-lane wave per 8x8 pixel block of a tile. A wave walks its
    tile's list back to front from the largest last contributor of its pixels and
    evaluates, on all 64 lanes, every entry at or before that position whose pixel box
    meets the block and whose least Mahalanobis distance m over the block's pixel
    centres is within min(ext^2, 2 ln(o / alpha_min)) (the kernel's staging tests,
    replayed here in FP64 without the kernel's rounding slack). Each such step also
    sums the nine gradient terms over the wave once.

    Returns {"steps" (= wave-Gaussian pairs, each one nine-value wave reduction),
    "lane_evaluations" (= 64 x steps), "algorithmic_evaluations" (every (pixel, list
    entry) pair up to the pixel's last contributor: the method's own count)}.
    """
    import torch
    T = cfg.tile_size
    nb = T // 8                                     # 8x8 blocks per tile side
    dev = st.ranges.device
    M = int(st.count.item())
    vals = st.vals[:M].long() & 0xFFFFFFFF
    tile = st.tile_ids(cfg)[:M].long()
    rec = st.record.view(-1, 12)[vals]
    lo = rec[:, 0].view(torch.int32).long()
    hi = rec[:, 1].view(torch.int32).long()
    ilo, jlo, ihi, jhi = lo & 0xFFFF, (lo >> 16) & 0xFFFF, hi & 0xFFFF, (hi >> 16) & 0xFFFF
    c0, c1 = rec[:, 2].double(), rec[:, 3].double()
    w00, w10, w11, opac = (rec[:, k].double() for k in (4, 5, 6, 7))
    del rec
    thr = torch.clamp(2.0 * (torch.log(opac) - math.log(cfg.alpha_min)), max=cfg.sigma_extent ** 2)
    pos = torch.arange(M, device=dev)
    ranges = st.ranges.view(-1, 2).long()
    toff = torch.tensor(st.tile_offset, device=dev)
    view = torch.searchsorted(toff, tile, right=True) - 1
    Wv = torch.tensor([c.width for c in st.cams], device=dev)[view]
    Hv = torch.tensor([c.height for c in st.cams], device=dev)[view]
    txn = (Wv + T - 1) // T
    lt = tile - toff[view]
    tx, ty = lt % txn, lt // txn
    # per (tile, 8x8 block): the largest last contributor of its pixels, capped at the
    # tile's last instance (-1 if no pixel blended anything)
    blk_last = torch.full((st.n_tiles, nb * nb), -1, dtype=torch.long, device=dev)
    algo = 0
    for v, cam in enumerate(st.cams):
        W, H = cam.width, cam.height
        txv, tyv = (W + T - 1) // T, (H + T - 1) // T
        last = st.view_plane(st.last_idx, v).long()
        pad = torch.full((tyv * T, txv * T), -1, dtype=torch.long, device=dev)
        pad[:H, :W] = last
        b8 = pad.view(tyv, nb, 8, txv, nb, 8).amax(dim=(2, 5))           # (tyv, nb, txv, nb)
        b8 = b8.permute(0, 2, 1, 3).reshape(tyv * txv, nb * nb)
        t0 = st.tile_offset[v]
        blk_last[t0:t0 + tyv * txv] = torch.minimum(b8, ranges[t0:t0 + tyv * txv, 1:2] - 1)
        # algorithmic: every list entry up to each pixel's last contributor
        tstart = ranges[t0:t0 + tyv * txv, 0].view(tyv, 1, txv, 1).expand(tyv, T, txv, T)
        tstart = tstart.reshape(tyv * T, txv * T)[:H, :W]
        algo += int(torch.clamp(last - tstart + 1, min=0).sum().item())
    ax = -c0 / w00                                  # the mean's offset from the corner centre
    ay = -(w10 * ax + c1) / w11
    steps = 0
    for b in range(nb * nb):
        bx, by = b % nb, b // nb
        x0, y0 = tx * T + 8 * bx, ty * T + 8 * by
        x1, y1 = torch.minimum(x0 + 7, Wv - 1), torch.minimum(y0 + 7, Hv - 1)
        ok = (x0 < Wv) & (y0 < Hv) & (ilo <= x1) & (ihi >= x0) & (jlo <= y1) & (jhi >= y0)
        xa, xb = (x0 - ilo).double(), (x1 - ilo).double()
        ya, yb = (y0 - jlo).double(), (y1 - jlo).double()

        def edge_x(X):      # least m on the edge Dx = X
            dj = torch.clamp(-(w10 * X + c1) / w11, min=ya, max=yb)
            return (w00 * X + c0) ** 2 + (w10 * X + w11 * dj + c1) ** 2

        def edge_y(Y):      # least m on the edge Dy = Y
            di = -(w00 * c0 + w10 * (w11 * Y + c1)) / (w00 ** 2 + w10 ** 2)
            di = torch.minimum(torch.maximum(di, xa), xb)
            return (w00 * di + c0) ** 2 + (w10 * di + w11 * Y + c1) ** 2

        inside = (ax >= xa) & (ax <= xb) & (ay >= ya) & (ay <= yb)
        mmin = torch.minimum(torch.minimum(edge_x(xa), edge_x(xb)),
                             torch.minimum(edge_y(ya), edge_y(yb)))
        mmin = torch.where(inside, torch.zeros_like(mmin), mmin)
        ok &= (mmin <= thr) & (pos <= blk_last[tile, b])
        steps += int(ok.sum().item())
    return {"steps": steps, "lane_evaluations": 64 * steps, "algorithmic_evaluations": algo}


def roofline(stages, state, count, n, V, cfg):
    """Roofline of the dominant kernel. For the backward blend (VALU bound): the lane
    evaluations the launch issues (backward_work) x the FP32 arithmetic of one
    evaluation (BWD_OPS_PER_EVAL), over the launch's event-timed duration, against the
    FP32 VALU peak; the method's own evaluation count beside it as
    ``algorithmic_frac``. For a streaming kernel: its algorithmic bytes over HBM peak."""
    ms = stages["ms"]
    dom = max(("render_fwd", "render_bwd", "project", "project_bwd", "sort"), key=lambda k: ms[k])
    st = stages["state"]
    if dom == "render_bwd":
        wk = backward_work(st, cfg)
        sec = ms[dom] * 1e-3
        achieved = wk["lane_evaluations"] * BWD_OPS_PER_EVAL / sec / 1e12
        algo = wk["algorithmic_evaluations"] * BWD_OPS_PER_EVAL / sec / 1e12
        return {"kernel": dom, "bound": "alu", "achieved": round(achieved, 3),
                "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s (FP32 VALU lane-ops)",
                "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": measured_traffic(dom),
                "duration_ms": round(ms[dom], 4),
                "units": {**wk, "ops_per_evaluation": BWD_OPS_PER_EVAL},
                "algorithmic_frac": round(algo / VALU_PEAK_TOPS, 4)}
    if dom == "render_fwd":
        return {"kernel": dom, "bound": "alu", "achieved": None, "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s (FP32 VALU lane-ops)", "frac": None, "traffic": None}
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
    36 B screen-space gradient (the kernel recomputes the projection: it reads no
    records).
    """
    from paper_2308_04079_amd import _lib
    vis = int((st.tiles_touched[:V * n] > 0).sum().item())
    par = 4 * (11 + 3 * K)
    tile_passes = -(-_lib.lib().gs_sort_key_bits(st.n_tiles) // digit_bits)
    depth_passes = -(-31 // digit_bits)
    b = {"project": par * n + 8 * V * n + 48 * vis,
         "bin": 4 * V * n + (12 + 16 * depth_passes) * vis + 8 * count,
         "sort": 16 * count * tile_passes,
         "project_bwd": 2 * par * n + 4 * V * n + 36 * vis}
    out = {}
    for k, v in b.items():
        gbs = v / (ms[k] * 1e-3) / 1e9
        out[k] = {"bytes": v, "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["bin"]["depth_passes"] = depth_passes
    out["sort"]["passes"] = tile_passes
    out["visible_pairs"] = vis
    return out


# FP32 VALU operations of one (pixel, Gaussian) evaluation of the backward blend, as the
# method states it (one op per add, mul, fma, compare, select, min, exp, reciprocal):
# about 40 arithmetic ops plus one exp and one reciprocal. The nine-value reduction of
# a step's gradients over the wave is its own unit (one per step), not counted per
# evaluation.
BWD_OPS_PER_EVAL = 42


# ---------------------------------------------------------------------------
# the FP64 oracle timed on the host cores (the reported CPU baseline)
# ---------------------------------------------------------------------------

_ORACLE = {}   # scene, projection and tile lists, shared with forked worker processes


def _oracle_gaussian_chunk(bounds):
    """Worker: projection and projection backward of one slice of the Gaussians (the
    per-Gaussian phases; their cost does not depend on the gradient values)."""
    from threadpoolctl import threadpool_limits

    from oracle.adjoint import empty_acc, project_backward
    from oracle.gaussians import project
    lo, hi = bounds
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        sub = _ORACLE["scene"].subset(slice(lo, hi))
        p = project(sub, _ORACLE["cam"], _ORACLE["rules"])
        if not _ORACLE["fwd_only"]:
            project_backward(sub, p, empty_acc(p.n))
        return time.perf_counter() - t


def _oracle_tile_chunk(tiles):
    """Worker: blend (forward, or forward + adjoint) of the listed tiles; returns the
    seconds of each."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.adjoint import blend_backward, empty_acc
    from oracle.raster import blend, tile_pixels
    p, tl, r = _ORACLE["proj"], _ORACLE["lists"], _ORACLE["rules"]
    cam = _ORACLE["cam"]
    out = []
    with threadpool_limits(limits=1):
        rng = np.random.default_rng(int(tiles[0]) if len(tiles) else 0)
        acc = empty_acc(p.n)
        for tt in tiles:
            t = time.perf_counter()
            px, py = tile_pixels(int(tt), tl, cam.width, cam.height, r.tile)
            ids = tl.ids[tl.start[tt]:tl.start[tt + 1]]
            if _ORACLE["fwd_only"]:
                blend(p, ids, px, py, r)
            else:
                blend_backward(p, ids, px, py, rng.standard_normal((len(px), 3)), r, acc)
            out.append(time.perf_counter() - t)
    return out


def stratified_tiles(lengths, n_sample, rng):
    """A seeded sample of n_sample tiles stratified by list length: the tiles sorted by
    length are cut into n_sample strata of (nearly) equal size and one tile is drawn
    from each; returns (tiles, stratum sizes). Sum over the sample of stratum size x
    per-tile cost estimates the frame's cost without bias, with far less variance than
    a plain random sample of the heavy-tailed tile costs."""
    import numpy as np
    order = np.argsort(lengths, kind="stable")
    edges = np.linspace(0, len(order), n_sample + 1).astype(np.int64)
    tiles, weights = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        if b > a:
            tiles.append(int(order[rng.integers(a, b)]))
            weights.append(int(b - a))
    return np.array(tiles, dtype=np.int64), np.array(weights, dtype=np.float64)


def oracle_view_seconds(sc, cam, procs, tiles_per_proc, fwd_only=False, seed=0):
    """Seconds the oracle takes for one view, on `procs` processes of one thread each.

    Per-Gaussian phases (projection, projection backward) are split over the processes
    by Gaussian slices; the tile lists (one global stable sort) run in one process; the
    blend is timed on a seeded sample of procs * tiles_per_proc tiles (every tile when
    the view has no more), stratified by list length, and scaled to the frame.
    Returns the phase times."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.gaussians import project
    from oracle.raster import tile_lists
    from oracle.rules import Rules
    r = Rules()
    _ORACLE.update(scene=sc, cam=cam, rules=r, fwd_only=fwd_only)
    ctx = mp.get_context("fork")
    bounds = np.linspace(0, sc.n, procs + 1).astype(np.int64)
    chunks = [(int(bounds[i]), int(bounds[i + 1])) for i in range(procs)]
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        if procs == 1:
            _oracle_gaussian_chunk(chunks[0])
        else:
            with ctx.Pool(procs) as pool:
                pool.map(_oracle_gaussian_chunk, chunks)
        t_gauss = time.perf_counter() - t
        p = project(sc, cam, r)           # the parent's copy for the lists and the blend
        t = time.perf_counter()
        tl = tile_lists(p, r)
        t_lists = time.perf_counter() - t
    _ORACLE.update(proj=p, lists=tl)
    n_tiles = tl.tiles_x * tl.tiles_y
    n_sample = min(n_tiles, procs * tiles_per_proc)
    sample, weight = stratified_tiles(np.diff(tl.start), n_sample,
                                      np.random.default_rng(seed))
    parts = [np.arange(i, len(sample), procs) for i in range(procs)]
    t = time.perf_counter()
    if procs == 1:
        per_tile = [_oracle_tile_chunk(sample)]
    else:
        with ctx.Pool(procs) as pool:
            per_tile = pool.map(_oracle_tile_chunk, [sample[k] for k in parts])
    t_tiles = time.perf_counter() - t
    _ORACLE.clear()
    secs = np.zeros(len(sample))
    for k, ts in zip(parts, per_tile):
        secs[k] = ts
    # frame estimate: the stratified sum of per-tile seconds, run at the parallel
    # efficiency the sample itself reached on `procs` processes
    frame_cpu = float((secs * weight).sum())
    t_blend = frame_cpu * t_tiles / max(float(secs.sum()), 1e-12) if procs > 1 else frame_cpu
    return {"per_gaussian_s": t_gauss, "lists_s": t_lists, "blend_sample_s": t_tiles,
            "blend_s": t_blend, "tiles_sampled": int(len(sample)), "tiles": int(n_tiles),
            "view_s": t_gauss + t_lists + t_blend}


def oracle_procs():
    """Worker processes for the multi-process oracle timing: one per host core, at most
    16 (the host share of one GPU)."""
    return max(1, min(os.cpu_count() or 1, 16))


def cpu_baseline(log):
    """The FP64 oracle on one view of the benchmark workload (3M Gaussians, 1920x1080,
    fwd+bwd), at one process and at one process per host core, each process holding
    NumPy's thread pools to one thread. ``value`` / ``cores`` are the multi-process
    figure; ``value_1_process`` the single-process one."""
    import scenes
    sc, cams = scenes.workload("train4")
    cam = cams[0]
    P = oracle_procs()
    one = oracle_view_seconds(sc, cam, 1, 48)
    log(f"[bench] oracle, 1 process: {one['view_s']:.0f} s per view "
        f"(per-Gaussian {one['per_gaussian_s']:.1f} s, lists {one['lists_s']:.1f} s, "
        f"{one['tiles_sampled']} tiles {one['blend_sample_s']:.1f} s)")
    multi = one
    if P > 1:
        multi = oracle_view_seconds(sc, cam, P, 16)
        log(f"[bench] oracle, {P} processes: {multi['view_s']:.0f} s per view "
            f"(per-Gaussian {multi['per_gaussian_s']:.1f} s, lists {multi['lists_s']:.1f} s, "
            f"{multi['tiles_sampled']} tiles {multi['blend_sample_s']:.1f} s)")
    return {"value": round(1.0 / multi["view_s"], 6), "unit": "views/s", "cores": P,
            "kind": "oracle",
            "value_1_process": round(1.0 / one["view_s"], 6),
            "sample": f"one 1920x1080 view of the 3M-Gaussian workload, fwd+bwd: projection and "
                      f"projection backward of every Gaussian split over {P} processes, tile "
                      f"lists in one, fwd+bwd blend of {multi['tiles_sampled']} seeded tiles of "
                      f"{multi['tiles']} (stratified by list length) scaled to the frame at "
                      f"the sample's parallel efficiency; value_1_process: the "
                      f"same in one process with {one['tiles_sampled']} tiles; NumPy FP64, "
                      f"one thread per process"}


def oracle_table(log):
    """The oracle per view on the parity workloads, at one process and at one process
    per host core: 1k Gaussians at 128x128 (forward only, every tile), 100k at 1280x720,
    3M at 1920x1080 and one 1920x1080 view of the 1M-Gaussian multi-view scene (fwd+bwd,
    sampled tiles)."""
    import scenes
    P = oracle_procs()
    rows = []
    for name, fwd_only in (("small", True), ("single720", False), ("full1080", False),
                           ("multiview", False)):
        sc, cams = scenes.workload(name)
        cam = cams[0]
        if name == "multiview":
            cam = next(c for c in cams if c.width == 1920)
        row = {"workload": name, "gaussians": sc.n, "resolution": f"{cam.width}x{cam.height}",
               "pass": "fwd" if fwd_only else "fwd+bwd", "processes": P}
        for procs in sorted({1, P}):
            t = oracle_view_seconds(sc, cam, procs, 48 if procs == 1 else 16, fwd_only)
            row[f"view_s_{procs}"] = round(t["view_s"], 3)
            row[f"tiles_sampled_{procs}"] = t["tiles_sampled"]
            log(f"[oracle] {name} {procs} process(es): {t['view_s']:.2f} s per view")
        rows.append(row)
    print(json.dumps({"oracle_seconds_per_view": rows, "host_cores": os.cpu_count()}), flush=True)


if __name__ == "__main__":
    main()
