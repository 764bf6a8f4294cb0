"""ctypes binding of libgs_mi355x.so: struct mirrors of include/gs.h and argument marshalling.

torch is imported before the library is loaded so that the library's HIP runtime
dependency (soname libamdhip64.so.7) resolves to the runtime torch already loaded,
and torch's stream handles are valid for it.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede the dlopen below)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgs_mi355x.so")

MAX_VIEWS = 32
RECORD_FLOATS = 12
GRAD2D_FLOATS = 9
MAX_INSTANCES = (1 << 30) - 1
STATUS_CAPACITY = 1
STATUS_SORT = 2

OK, ERR_ARG, ERR_CAPACITY, ERR_HIP, ERR_UNSUPPORTED, ERR_SORT, ERR_SCRATCH = 0, -1, -2, -3, -4, -5, -6
SORT_SCRATCH_BYTES = 16 << 20

c_float_p = ctypes.c_void_p


class GsCamera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class GsConfig(ctypes.Structure):
    _fields_ = [("sh_degree", ctypes.c_int32), ("tile_size", ctypes.c_int32),
                ("near_z", ctypes.c_float), ("sigma_extent", ctypes.c_float),
                ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("T_min", ctypes.c_float), ("bg", ctypes.c_float * 3),
                ("sort_digit_bits", ctypes.c_int32), ("lds_batch", ctypes.c_int32),
                ("isotropic", ctypes.c_int32), ("grad_limit", ctypes.c_int32)]


class GsParams(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p),
                ("sh", ctypes.c_void_p), ("n", ctypes.c_int64)]


class GsParamsGrad(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p),
                ("sh", ctypes.c_void_p)]


class GsProjected(ctypes.Structure):
    _fields_ = [("depth_key", ctypes.c_void_p), ("tiles_touched", ctypes.c_void_p),
                ("record", ctypes.c_void_p)]


class GsInstances(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("vals", ctypes.c_void_p),
                ("keys_alt", ctypes.c_void_p), ("vals_alt", ctypes.c_void_p),
                ("capacity", ctypes.c_int64), ("count", ctypes.c_void_p),
                ("status", ctypes.c_void_p)]


class GsDensifyConfig(ctypes.Structure):
    _fields_ = [("grad_threshold", ctypes.c_float), ("min_opacity", ctypes.c_float),
                ("split_scale", ctypes.c_float), ("max_world_scale", ctypes.c_float),
                ("max_screen_radius", ctypes.c_float), ("split_factor", ctypes.c_float)]


P = ctypes.POINTER
EXPORTS = {
    "gs_default_config": (None, [P(GsConfig)]),
    "gs_tile_layout": (ctypes.c_int64, [P(GsCamera), ctypes.c_int32, ctypes.c_int32,
                                        P(ctypes.c_int64)]),
    "gs_sort_key_bits": (ctypes.c_int32, [ctypes.c_int64]),
    "gs_project": (ctypes.c_int, [P(GsParams), P(GsCamera), ctypes.c_int32, P(GsConfig),
                                  P(GsProjected), ctypes.c_void_p]),
    "gs_bin_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, P(GsConfig)]),
    "gs_sorted_tile_ids": (ctypes.c_void_p, [P(GsInstances), ctypes.c_int64, P(GsConfig)]),
    "gs_bin": (ctypes.c_int, [P(GsProjected), ctypes.c_int64, P(GsCamera), ctypes.c_int32,
                              P(GsConfig), P(GsInstances), ctypes.c_void_p, ctypes.c_size_t,
                              ctypes.c_void_p]),
    "gs_sort_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64, P(GsConfig)]),
    "gs_sort": (ctypes.c_int, [P(GsInstances), ctypes.c_int64, P(GsConfig), ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                               ctypes.c_void_p]),
    "gs_sort_noalloc": (ctypes.c_int, [P(GsInstances), ctypes.c_int64, P(GsConfig),
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gs_render_fwd": (ctypes.c_int, [P(GsProjected), P(GsInstances), ctypes.c_void_p,
                                     ctypes.c_void_p, P(GsCamera), ctypes.c_int32, P(GsConfig),
                                     ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p]),
    "gs_render_bwd": (ctypes.c_int, [P(GsProjected), P(GsInstances), ctypes.c_void_p,
                                     ctypes.c_void_p, P(GsCamera), ctypes.c_int32, P(GsConfig),
                                     ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int64, ctypes.c_void_p]),
    "gs_render_l1_workspace_bytes": (ctypes.c_size_t, [P(GsCamera), ctypes.c_int32,
                                                      P(GsConfig)]),
    "gs_render_bwd_l1": (ctypes.c_int, [P(GsProjected), P(GsInstances), ctypes.c_void_p,
                                        ctypes.c_void_p, P(GsCamera), ctypes.c_int32,
                                        P(GsConfig), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_int64, ctypes.c_void_p]),
    "gs_project_bwd": (ctypes.c_int, [P(GsParams), P(GsCamera), ctypes.c_int32, P(GsConfig),
                                      P(GsProjected), ctypes.c_void_p, P(GsParamsGrad),
                                      ctypes.c_void_p]),
    "gs_loss_workspace_bytes": (ctypes.c_size_t, [P(GsCamera), ctypes.c_int32]),
    "gs_loss_photometric": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, P(GsCamera),
                                           ctypes.c_int32, ctypes.c_float, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_void_p]),
    "gs_loss_l1": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, P(GsCamera), ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gs_default_densify_config": (None, [P(GsDensifyConfig)]),
    "gs_densify_accumulate": (ctypes.c_int, [P(GsProjected), ctypes.c_void_p, P(GsCamera),
                                             ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gs_densify_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
    "gs_densify_plan": (ctypes.c_int, [P(GsParams), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, P(GsDensifyConfig), ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p]),
    "gs_densify_apply": (ctypes.c_int, [P(GsParams), ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, P(GsDensifyConfig),
                                        P(GsParamsGrad), ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "gs_densify_gather": (ctypes.c_int, [P(GsParams), ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int32, P(GsParamsGrad),
                                         ctypes.c_int64, ctypes.c_void_p]),
    "gs_adam_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_int32, ctypes.c_void_p]),
    "gs_reset_opacity": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_float,
                                        ctypes.c_void_p]),
    "gs_read_status": (ctypes.c_int, [P(GsInstances), P(ctypes.c_uint32), P(ctypes.c_uint32),
                                      ctypes.c_void_p]),
    "gs_status_string": (ctypes.c_char_p, [ctypes.c_int]),
}

_LIB = None


class GsError(RuntimeError):
    def __init__(self, fn, code):
        self.code = code
        super().__init__(f"{fn} failed: {code} ({status_string(code)})")


def lib():
    """The loaded library; raises if it has not been built (there is no fallback path)."""
    global _LIB
    if _LIB is None:
        # GS_LIBRARY: another build of the same library (e.g. to compare two builds)
        path = os.environ.get("GS_LIBRARY", LIB_PATH)
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with "
                               "`python -m paper_2308_04079_amd.build` (hipcc, gfx950)")
        h = ctypes.CDLL(path)
        for name, (res, args) in EXPORTS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _LIB = h
    return _LIB


def status_string(code: int) -> str:
    return lib().gs_status_string(int(code)).decode()


def check(fn: str, code: int):
    if code != OK:
        raise GsError(fn, code)


def ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def make_camera(cam) -> GsCamera:
    c = GsCamera()
    R = [float(x) for x in list(getattr(cam.R, "ravel", lambda: cam.R)())]
    t = [float(x) for x in list(getattr(cam.t, "ravel", lambda: cam.t)())]
    c.R[:] = R
    c.t[:] = t
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def make_cameras(cams):
    arr = (GsCamera * len(cams))()
    for k, cam in enumerate(cams):
        arr[k] = make_camera(cam)
    return arr


def default_config(**overrides) -> GsConfig:
    cfg = GsConfig()
    lib().gs_default_config(ctypes.byref(cfg))
    for k, v in overrides.items():
        if k == "bg":
            cfg.bg[:] = [float(x) for x in v]
        else:
            setattr(cfg, k, v)
    return cfg
