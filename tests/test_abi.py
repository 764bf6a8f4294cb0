"""The C ABI library loads on the CPU and exports every entry point include/gs.h declares.

No compute call is made here (there is no GPU): only the host-side helpers and the
argument checks that return before any HIP call.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(gs_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2308_04079_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libgs_mi355x.so is not built (run __graft_entry__.build())")
    return _lib


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 13, names
    h = L.lib()
    for name in names:
        assert hasattr(h, name), name
        assert name in L.EXPORTS, f"{name} is not bound in _lib.EXPORTS"


def test_binding_covers_only_declared_symbols(L):
    assert set(L.EXPORTS) <= set(declared_functions())


def test_struct_sizes_match_the_header_layout(L):
    assert ctypes.sizeof(L.GsCamera) == 4 * 18
    assert ctypes.sizeof(L.GsConfig) == 4 * 14
    assert ctypes.sizeof(L.GsParams) == 8 * 6
    assert ctypes.sizeof(L.GsInstances) == 8 * 7


def test_default_config_is_the_papers_rules(L):
    c = L.default_config()
    assert (c.sh_degree, c.tile_size, c.sort_digit_bits, c.lds_batch) == (3, 16, 8, 64)
    assert abs(c.near_z - 0.2) < 1e-7 and c.sigma_extent == 3.0
    assert abs(c.alpha_min - 1 / 255) < 1e-9 and abs(c.alpha_max - 0.99) < 1e-7
    assert abs(c.T_min - 1e-4) < 1e-10 and list(c.bg) == [0.0, 0.0, 0.0]
    assert (c.isotropic, c.grad_limit) == (0, 0)   # the method, not its ablations


def test_tile_layout_and_key_bits(L):
    import scenes
    cams = [scenes.pinhole_camera(1920, 1080), scenes.pinhole_camera(37, 29)]
    cc = L.make_cameras(cams)
    off = (ctypes.c_int64 * 3)()
    n = L.lib().gs_tile_layout(cc, 2, 16, off)
    assert list(off) == [0, 120 * 68, 120 * 68 + 3 * 2] and n == off[2]
    assert L.lib().gs_sort_key_bits(8160) == 13
    assert L.lib().gs_sort_key_bits(64) == 6
    assert L.lib().gs_sort_key_bits(1) == 0
    assert L.lib().gs_tile_layout(cc, 2, 12, None) == L.ERR_ARG
    assert L.lib().gs_tile_layout(cc, 0, 16, None) == L.ERR_ARG


def test_host_argument_checks_return_before_any_launch(L):
    import scenes
    lib = L.lib()
    cc = L.make_cameras([scenes.pinhole_camera(64, 64)])
    cfg = L.default_config()
    bad = L.default_config(sh_degree=5)
    for k, v in (("isotropic", 2), ("grad_limit", -1), ("lds_batch", 96), ("tile_size", 12)):
        b = L.default_config(**{k: v})
        assert lib.gs_project(ctypes.byref(L.GsParams(0, 0, 0, 0, 0, 10)), cc, 1, ctypes.byref(b),
                              ctypes.byref(L.GsProjected(0, 0, 0)), None) == L.ERR_ARG, k
    p = L.GsParams(0, 0, 0, 0, 0, 10)
    proj = L.GsProjected(0, 0, 0)
    assert lib.gs_project(ctypes.byref(p), cc, 1, ctypes.byref(bad), ctypes.byref(proj), None) == L.ERR_ARG
    assert lib.gs_project(ctypes.byref(p), cc, 1, ctypes.byref(cfg), ctypes.byref(proj), None) == L.ERR_ARG
    neg = L.GsParams(0, 0, 0, 0, 0, -1)
    assert lib.gs_project(ctypes.byref(neg), cc, 1, ctypes.byref(cfg), ctypes.byref(proj), None) == L.ERR_ARG
    many = L.make_cameras([scenes.pinhole_camera(8, 8)] * 33)
    inst = L.GsInstances(0, 0, 0, 0, 0, 0, 0)
    assert lib.gs_bin(ctypes.byref(proj), 1, many, 33, ctypes.byref(cfg), ctypes.byref(inst), None, 0, None) in (L.ERR_ARG, L.ERR_UNSUPPORTED)
    huge = L.make_cameras([scenes.pinhole_camera(40000, 8)])
    assert lib.gs_render_fwd(ctypes.byref(proj), ctypes.byref(inst), 1, None, huge, 1, ctypes.byref(cfg), 1, 1, 1, 1, None) == L.ERR_UNSUPPORTED
    assert lib.gs_sort(ctypes.byref(inst), 10, ctypes.byref(cfg), None, None, None, 0, None) == L.ERR_ARG
    # the static-scratch sort: the same argument checks, then its size limit, all before
    # any device call (the pointers below are never dereferenced)
    assert lib.gs_sort_noalloc(ctypes.byref(inst), 10, ctypes.byref(cfg), None, None, None) == L.ERR_ARG
    fake = L.GsInstances(16, 16, 16, 16, 1 << 27, 16, 16)
    assert lib.gs_sort_workspace_bytes(1 << 27, 8160, ctypes.byref(cfg)) > L.SORT_SCRATCH_BYTES
    assert lib.gs_sort_noalloc(ctypes.byref(fake), 8160, ctypes.byref(cfg), 16, None, None) == L.ERR_SCRATCH
    fake.capacity = 1 << 30
    assert lib.gs_sort_noalloc(ctypes.byref(fake), 8160, ctypes.byref(cfg), 16, None, None) == L.ERR_UNSUPPORTED
    assert lib.gs_sort_noalloc(ctypes.byref(fake), 8160, ctypes.byref(bad), 16, None, None) == L.ERR_ARG
    assert lib.gs_status_string(L.ERR_SCRATCH) == b"needs more than the library's static scratch"
    # one set of per-block digit counts shared by the passes (256 words per 3072 keys)
    # and the digit totals, then the tile-order table (33 buckets per 1024 tiles)
    blocks = -(-(1 << 20) // 3072)
    counts = (256 * blocks + 256) * 4
    assert lib.gs_sort_workspace_bytes(1 << 20, 8160, ctypes.byref(cfg)) == \
        ((counts + 255) // 256) * 256 + (8160 + 1023) // 1024 * 33 * 4
    assert lib.gs_sort_key_bits(8160) == 13 and lib.gs_sort_key_bits(1) == 0
    assert lib.gs_bin_workspace_bytes(1000, ctypes.byref(cfg)) > 0
    assert lib.gs_bin_workspace_bytes(1000, ctypes.byref(bad)) == 0
    assert lib.gs_status_string(L.ERR_CAPACITY) == b"instance count exceeds capacity"


def test_densify_defaults_and_argument_checks(L):
    lib = L.lib()
    d = L.GsDensifyConfig()
    lib.gs_default_densify_config(ctypes.byref(d))
    assert (round(d.grad_threshold, 7), round(d.min_opacity, 6), round(d.split_factor, 5)) == (0.0002, 0.005, 1.6)
    assert d.max_world_scale == 0.0 and d.max_screen_radius == 0.0
    p = L.GsParams(0, 0, 0, 0, 0, 10)
    bad = L.GsDensifyConfig()
    lib.gs_default_densify_config(ctypes.byref(bad))
    bad.split_factor = 1.0
    n_out = ctypes.c_uint32(0)
    ws = ctypes.create_string_buffer(64)
    args = (None, None, None)
    assert lib.gs_densify_plan(ctypes.byref(p), *args, ctypes.byref(bad), None, None,
                               ctypes.byref(n_out), ws, 64, None) == L.ERR_ARG
    assert lib.gs_densify_plan(ctypes.byref(p), *args, ctypes.byref(d), None, None,
                               ctypes.byref(n_out), ws, 64, None) == L.ERR_ARG
    assert lib.gs_densify_workspace_bytes(-1) == 0
    assert lib.gs_densify_workspace_bytes(4096 * 3 + 1) == 5 * 4
    assert lib.gs_reset_opacity(None, 10, 1.5, None) == L.ERR_ARG
    assert lib.gs_reset_opacity(None, 10, 0.01, None) == L.ERR_ARG
    assert lib.gs_reset_opacity(None, 0, 0.01, None) == L.OK
    out = L.GsParamsGrad(0, 0, 0, 0, 0)
    assert lib.gs_densify_apply(ctypes.byref(p), 4, None, None, None, ctypes.byref(d),
                                ctypes.byref(out), 5, None, None) == L.ERR_ARG
    assert lib.gs_densify_apply(ctypes.byref(p), 1, None, None, None, ctypes.byref(d),
                                ctypes.byref(out), 5, None, None) == L.ERR_ARG


def test_loss_argument_checks(L):
    import scenes
    lib = L.lib()
    cc = L.make_cameras([scenes.pinhole_camera(40, 30)])
    assert lib.gs_loss_workspace_bytes(cc, 1) == 9 * 40 * 30 * 4
    ws = ctypes.create_string_buffer(16)
    assert lib.gs_loss_photometric(1, 1, cc, 1, 1.5, 1, None, ws, 16, None) == L.ERR_ARG
    assert lib.gs_loss_photometric(1, 1, cc, 1, 0.2, 1, None, ws, 16, None) == L.ERR_ARG
    assert lib.gs_loss_photometric(None, 1, cc, 1, 0.2, 1, None, ws, 16, None) == L.ERR_ARG


def test_fused_l1_backward_argument_checks(L):
    """gs_render_bwd_l1: one workspace float per 8x8 block of every tile; missing inputs
    or (with a loss) a missing or short workspace are refused before any launch."""
    import scenes
    lib = L.lib()
    cc = L.make_cameras([scenes.pinhole_camera(40, 30), scenes.pinhole_camera(17, 9)])
    for ts, tiles in ((8, 5 * 4 + 3 * 2), (16, 3 * 2 + 2 * 1), (32, 2 * 1 + 1 * 1)):
        cfg = L.default_config(tile_size=ts)
        assert lib.gs_render_l1_workspace_bytes(cc, 2, ctypes.byref(cfg)) == tiles * (ts // 8) ** 2 * 4
    assert lib.gs_render_l1_workspace_bytes(cc, 2, ctypes.byref(L.default_config(tile_size=12))) == 0
    assert lib.gs_render_l1_workspace_bytes(cc, 0, ctypes.byref(L.default_config())) == 0
    cfg = L.default_config()
    need = lib.gs_render_l1_workspace_bytes(cc, 2, ctypes.byref(cfg))
    proj = L.GsProjected(16, 16, 16)
    inst = L.GsInstances(16, 16, 16, 16, 64, 16, 16)
    ws = ctypes.create_string_buffer(need)
    head = (ctypes.byref(proj), ctypes.byref(inst), 16, None, cc, 2, ctypes.byref(cfg), 16, 16)
    # the pointers are never dereferenced: every call below fails its host checks
    assert lib.gs_render_bwd_l1(*head, None, 16, 16, 16, ws, need, 10, None) == L.ERR_ARG
    assert lib.gs_render_bwd_l1(*head, 16, None, 16, 16, ws, need, 10, None) == L.ERR_ARG
    assert lib.gs_render_bwd_l1(*head, 16, 16, None, 16, ws, need, 10, None) == L.ERR_ARG
    assert lib.gs_render_bwd_l1(*head, 16, 16, 16, 16, None, need, 10, None) == L.ERR_ARG
    assert lib.gs_render_bwd_l1(*head, 16, 16, 16, 16, ws, need - 4, 10, None) == L.ERR_ARG


def test_a_missing_library_fails_loudly():
    """No fallback: without the built library every entry raises."""
    import subprocess
    import sys
    code = ("import pytest\nfrom paper_2308_04079_amd import _lib\n"
            "with pytest.raises(RuntimeError, match='missing'):\n    _lib.lib()\nprint('raised')\n")
    env = dict(os.environ, GS_LIBRARY=os.path.join(ROOT, "no_such_library.so"))
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 0 and "raised" in out.stdout, out.stderr
