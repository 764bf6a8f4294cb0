"""Shared helpers of the GPU parity tests: run the HIP path, fetch its outputs as NumPy,
and compare them with the oracle."""
from __future__ import annotations

import numpy as np

from oracle.raster import pixel_outcomes
from oracle.rules import Rules

TOL_IMAGE = 1e-4      # max-abs image error (the benchmark spec)
TOL_GRAD = 1e-3       # relative L2 error per parameter group
TOL_GRAD_ELEM = 1e-3  # per element: |gpu - oracle| <= this x the group's largest |oracle|
AMBIGUOUS_MAX = 1e-3  # largest fraction of pixels with a decision within its margin
GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def gpu_render(scene, cams, **cfg):
    import torch
    from paper_2308_04079_amd import GaussianParams, Rasterizer
    params = GaussianParams.from_numpy(scene, "cuda")
    rast = Rasterizer(sh_degree=scene.sh_degree, **cfg)
    state = rast.render(params, cams)
    torch.cuda.synchronize()
    return rast, params, state


def to_np(t):
    return t.detach().cpu().numpy()


def gpu_images(state):
    """Per view: (image HxWx3 float64, T_final HxW, last Gaussian id HxW or -1)."""
    vals = to_np(state.vals).astype(np.int64) & 0xFFFFFFFF
    out = []
    for v in range(state.n_views):
        img = to_np(state.view_image(v)).transpose(1, 2, 0).astype(np.float64)
        T = to_np(state.view_plane(state.T_final, v)).astype(np.float64)
        last = to_np(state.view_plane(state.last_idx, v)).astype(np.int64)
        gid = np.where(last >= 0, vals[np.maximum(last, 0)] - v * state.n, -1)
        out.append((img, T, gid))
    return out


def T_tolerance(T_ref, T_err):
    """Allowed |T_gpu - T_oracle|: the oracle's first-order bound on the FP32 rounding of
    the running product (relative T_err), plus one rounding of the stored value."""
    return T_ref * (T_err + 2.0 ** -24)


def check_view_image(gpu, proj, ref, tl, rules: Rules = Rules()):
    """Image parity of one view on the pixels the oracle rendered (ref.done).

    Pixels whose decisions all lie outside their margins: colour within TOL_IMAGE,
    T_final within its rounding bound, the same last contributor. Pixels with a
    decision within its margin: the GPU result must equal one of the legitimate
    outcomes, i.e. the oracle re-run with any combination of those decisions taken
    the other way. Returns counts for reporting."""
    img, T, gid = gpu
    done = ref.done
    amb = done & ref.ambiguous
    n_done = int(done.sum())
    assert amb.sum() <= AMBIGUOUS_MAX * n_done, (int(amb.sum()), n_done)
    m = done & ~ref.ambiguous
    err = np.abs(img - ref.color)[m]
    worst = float(err.max()) if err.size else 0.0
    assert worst <= TOL_IMAGE, worst
    bad_T = np.abs(T - ref.T_final) > T_tolerance(ref.T_final, ref.T_err)
    assert not np.any(bad_T & m), (int((bad_T & m).sum()),
                                   float(np.max(np.abs(T / ref.T_final - 1)[m])))
    assert np.array_equal(gid[m], ref.last_id[m])
    flipped = 0
    for y, x in zip(*np.nonzero(amb)):
        t = (y // rules.tile) * tl.tiles_x + x // rules.tile
        ids = tl.ids[tl.start[t]:tl.start[t + 1]]
        outs = pixel_outcomes(proj, ids, int(x), int(y), rules)
        match = [k for k, o in enumerate(outs)
                 if np.abs(img[y, x] - o.color[0]).max() <= TOL_IMAGE
                 and abs(T[y, x] - o.T_final[0]) <= T_tolerance(o.T_final[0], o.T_err[0])
                 and gid[y, x] == o.last_id[0]]
        assert match, (int(x), int(y), img[y, x], [o.color[0] for o in outs])
        flipped += 0 not in match
    return {"pixels": n_done, "ambiguous": int(amb.sum()), "other_branch": flipped,
            "worst": worst}


def check_grads(grads, gref, groups=GROUPS):
    """Per group: relative L2 within TOL_GRAD, and every element within TOL_GRAD_ELEM of
    the group's largest oracle magnitude (a systematic error on a few Gaussians
    cannot hide under the norm)."""
    for k in groups:
        a = np.asarray(grads[k], dtype=np.float64)
        b = np.asarray(gref[k], dtype=np.float64)
        r = rel_l2(a, b)
        assert r <= TOL_GRAD, (k, r)
        scale = float(np.abs(b).max()) if b.size else 0.0
        d = float(np.abs(a - b).max()) if b.size else 0.0
        assert d <= TOL_GRAD_ELEM * scale + 1e-30, (k, d, scale)


def decode_records(state, v):
    """GPU projection of view v: dict of per-Gaussian arrays."""
    n = state.n
    tt = to_np(state.tiles_touched)[v * n:(v + 1) * n]
    dk = to_np(state.depth_key)[v * n:(v + 1) * n].view(np.uint32)
    rec = to_np(state.record).reshape(-1, 12)[v * n:(v + 1) * n]
    lo = rec[:, 0].view(np.int32)
    hi = rec[:, 1].view(np.int32)
    i_lo, j_lo = lo & 0xFFFF, (lo >> 16) & 0xFFFF
    i_hi, j_hi = hi & 0xFFFF, (hi >> 16) & 0xFFFF
    w00, w10, w11 = (rec[:, k].astype(np.float64) for k in (4, 5, 6))
    c0, c1 = rec[:, 2].astype(np.float64), rec[:, 3].astype(np.float64)
    # Q = W^T W with W = [[w00, 0], [w10, w11]]
    Q = np.empty((n, 2, 2))
    Q[:, 0, 0] = w00 * w00 + w10 * w10
    Q[:, 0, 1] = Q[:, 1, 0] = w10 * w11
    Q[:, 1, 1] = w11 * w11
    # c = W (corner centre - mean): the mean is the corner centre minus W^-1 c
    with np.errstate(all="ignore"):
        ax = c0 / w00
        ay = (c1 - w10 * ax) / w11
    return dict(valid=tt > 0, tiles=tt, zkey=dk, i_lo=i_lo, i_hi=i_hi, j_lo=j_lo, j_hi=j_hi,
                u=i_lo + 0.5 - ax, v=j_lo + 0.5 - ay,
                conic=Q, opacity=rec[:, 7].astype(np.float64),
                rgb=rec[:, 8:11].astype(np.float64), w=rec[:, 4:7].astype(np.float64))


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / max(nb, 1e-30)
