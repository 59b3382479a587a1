"""The C-ABI library loads and exports every symbol include/pvg.h declares,
and host-side argument validation rejects bad calls before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(pvg_\w+)\s*\(", src, re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2311_18561_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpvg.so is not built (python -m paper_2311_18561_amd.build)")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    from paper_2311_18561_amd import _lib as L
    assert L.status_str(0) == "ok"
    assert "capacity" in L.status_str(L.PVG_ERR_CAPACITY)


def test_invalid_arguments_rejected_on_host(lib):
    from paper_2311_18561_amd import _lib as L
    g = L.Gaussians()
    g.n = -1
    cam = L.Camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.znear = 64, 48, 50.0, 50.0, 0.2
    fr = L.Frame()
    geom = L.Geom()
    assert lib.pvg_preprocess(C.byref(g), C.byref(cam), C.byref(fr), C.byref(geom), None) == L.PVG_ERR_INVALID
    assert "n = -1" in L.last_error()
    g.n = 10
    g.sh_degree = 4
    assert lib.pvg_preprocess(C.byref(g), C.byref(cam), C.byref(fr), C.byref(geom), None) == L.PVG_ERR_INVALID
    g.sh_degree = 0
    assert lib.pvg_preprocess(C.byref(g), C.byref(cam), C.byref(fr), C.byref(geom), None) == L.PVG_ERR_INVALID
    assert lib.pvg_preprocess(None, C.byref(cam), C.byref(fr), C.byref(geom), None) == L.PVG_ERR_INVALID
    cam.fx = 0.0
    g.n = 0
    assert lib.pvg_preprocess(C.byref(g), C.byref(cam), C.byref(fr), C.byref(geom), None) == L.PVG_ERR_INVALID
    bins = L.Bins()
    bins.capacity = -5
    cam.fx = 50.0
    assert lib.pvg_bin_sort(C.byref(geom), C.byref(cam), C.byref(bins), None, 0, 1, None) == L.PVG_ERR_INVALID
    fr.advect_mode = 3
    assert lib.pvg_render_fwd(C.byref(geom), C.byref(bins), C.byref(cam), C.byref(fr), None, None, None,
                              None) == L.PVG_ERR_INVALID
    # a near plane at or behind the camera is rejected (depth keys need z > 0)
    fr.advect_mode = 0
    for z in (0.0, -1.0, float("nan")):
        cam.znear = z
        assert lib.pvg_preprocess(C.byref(g), C.byref(cam), C.byref(fr), C.byref(geom), None) == L.PVG_ERR_INVALID
        assert "znear" in L.last_error()
    cam.znear = 0.2
    # list form flag and the multi-view adjoint's arguments
    bins.capacity = 0
    bins.ranges = bins.counters = 1
    bins.tile_cull = 2
    assert lib.pvg_bin_sort(C.byref(geom), C.byref(cam), C.byref(bins), None, 0, 1, None) == L.PVG_ERR_INVALID
    assert "tile_cull" in L.last_error()
    gg = L.GaussiansGrad()
    assert lib.pvg_render_bwd_views(C.byref(g), 0, C.byref(cam), C.byref(fr), C.byref(geom), C.byref(bins), None,
                                    None, None, C.byref(gg), 0, None, 0, None) == L.PVG_ERR_INVALID
    size = C.c_size_t()
    assert lib.pvg_bwd_views_tmp_bytes(100, 6, 64, 48, 1000, C.byref(size)) == 0 and size.value > 0
    assert lib.pvg_bwd_views_tmp_bytes(100, 0, 64, 48, 1000, C.byref(size)) == L.PVG_ERR_INVALID
    # the sky composite: null arrays and the cube resolution
    cam.znear = 0.2
    assert lib.pvg_sky_composite(C.byref(cam), None, None, None, 8, None, None, None) == L.PVG_ERR_INVALID
    assert lib.pvg_sky_composite(C.byref(cam), 1, 1, 1, 0, None, 1, None) == L.PVG_ERR_INVALID
    assert "cube_res" in L.last_error()
    assert lib.pvg_sky_composite_bwd(C.byref(cam), 1, 1, 1, 20000, None, 1, 1, None) == L.PVG_ERR_INVALID
    # the multi-view preprocess: view count, null arrays, a bad camera among the views
    g.n, g.sh_degree = 0, 0
    cams2 = (L.Camera * 2)(cam, cam)
    frs2 = (L.Frame * 2)(fr, fr)
    geoms2 = (L.Geom * 2)(geom, geom)
    assert lib.pvg_preprocess_views(C.byref(g), 0, cams2, frs2, geoms2, None) == L.PVG_ERR_INVALID
    assert lib.pvg_preprocess_views(C.byref(g), 2, cams2, None, geoms2, None) == L.PVG_ERR_INVALID
    cams2[1].znear = 0.0
    assert lib.pvg_preprocess_views(C.byref(g), 2, cams2, frs2, geoms2, None) == L.PVG_ERR_INVALID
    assert "znear" in L.last_error()


def test_workspace_query(lib):
    from paper_2311_18561_amd import _lib as L
    ws = L.WsSizes()
    assert lib.pvg_workspace_query(1000, 128, 96, 10000, C.byref(ws)) == 0
    assert ws.num_tiles == 48 and ws.bin_tmp_bytes > 0 and ws.bwd_tmp_bytes >= 1000 * 12 * 4
    assert lib.pvg_workspace_query(1000, 100, 70, 0, C.byref(ws)) == 0
    assert ws.num_tiles == 7 * 5
    assert lib.pvg_workspace_query(-1, 128, 96, 0, C.byref(ws)) == L.PVG_ERR_INVALID


def test_new_entry_points_reject_bad_arguments_on_host(lib):
    """The adaptive control, optimizer, SSIM and staticness entry points
    validate on the host before any launch."""
    from paper_2311_18561_amd import _lib as L
    size = C.c_size_t()
    assert lib.pvg_densify_tmp_bytes(-1, C.byref(size)) == L.PVG_ERR_INVALID
    assert lib.pvg_densify_tmp_bytes((1 << 30) + 1, C.byref(size)) == L.PVG_ERR_INVALID
    assert lib.pvg_densify_tmp_bytes(1000, C.byref(size)) == 0 and size.value >= 1000
    g = L.Gaussians()
    g.n, g.sh_degree = 0, 0
    n_out = C.c_int64()
    bad = L.DensifyConfig(1.7e-4, 0.0, 0.3, 3.0, 0.0, 0.8, 1.0)  # r = 0
    assert lib.pvg_densify_plan(C.byref(g), None, None, None, C.byref(bad), 1, 1 << 20, C.byref(n_out),
                                None) == L.PVG_ERR_INVALID
    assert "scene_radius" in L.last_error()
    bad.scene_radius, bad.clone_scale = 30.0, float("inf")
    assert lib.pvg_densify_plan(C.byref(g), None, None, None, C.byref(bad), 1, 1 << 20, C.byref(n_out),
                                None) == L.PVG_ERR_INVALID
    g.n = 10
    ok = L.DensifyConfig(1.7e-4, 30.0, 0.3, 3.0, 0.0, 0.8, 1.0)
    g.mu = g.scale = g.rot = g.sh = g.opacity = g.vel = g.period = g.tau = g.beta = 1
    assert lib.pvg_densify_plan(C.byref(g), None, 1, 1, C.byref(ok), 1, 1 << 20, C.byref(n_out),
                                None) == L.PVG_ERR_INVALID  # statistics missing
    assert lib.pvg_densify_plan(C.byref(g), 1, 1, 1, C.byref(ok), 1, 4, C.byref(n_out), None) == L.PVG_ERR_NOMEM
    # Adam: step >= 1, betas in [0, 1), eps > 0, rates finite and >= 0
    cfg = L.AdamConfig()
    cfg.beta1, cfg.beta2, cfg.eps, cfg.step = 0.9, 0.999, 1e-15, 0
    gg = L.GaussiansGrad()
    assert lib.pvg_adam_step(C.byref(g), C.byref(gg), 1, 1, C.byref(cfg), None) == L.PVG_ERR_INVALID
    cfg.step, cfg.beta1 = 1, 1.0
    assert lib.pvg_adam_step(C.byref(g), C.byref(gg), 1, 1, C.byref(cfg), None) == L.PVG_ERR_INVALID
    cfg.beta1, cfg.lr[3] = 0.9, -1e-3
    assert lib.pvg_adam_step(C.byref(g), C.byref(gg), 1, 1, C.byref(cfg), None) == L.PVG_ERR_INVALID
    cfg.lr[3] = 1e-3
    assert lib.pvg_adam_step(C.byref(g), C.byref(gg), 1, 1, C.byref(cfg), None) == L.PVG_ERR_INVALID  # grads null
    assert lib.pvg_opacity_reset(C.byref(g), 1, 1, float("nan"), None) == L.PVG_ERR_INVALID
    # SSIM: sizes and arrays
    assert lib.pvg_ssim_fwd(1, 1, 3, 0, 16, None, 1, None) == L.PVG_ERR_INVALID
    assert lib.pvg_ssim_fwd(None, 1, 3, 16, 16, None, 1, None) == L.PVG_ERR_INVALID
    assert lib.pvg_ssim_bwd(1, 1, 1, None, 3, 16, 16, 1, None) == L.PVG_ERR_INVALID
    # staticness split: threshold and workspace
    assert lib.pvg_staticness_split_plan(C.byref(g), float("nan"), 1, 1 << 20, C.byref(n_out),
                                         None) == L.PVG_ERR_INVALID
    assert lib.pvg_staticness_split_plan(C.byref(g), 0.5, 1, 4, C.byref(n_out), None) == L.PVG_ERR_NOMEM
    # the densify statistics go as a pair
    gg.mu = gg.scale = gg.rot = gg.sh = gg.opacity = gg.vel = gg.period = gg.tau = gg.beta = 1
    gg.densify_grad = 1
    cam = L.Camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.znear = 64, 48, 50.0, 50.0, 0.2
    fr = L.Frame()
    geom, bins = L.Geom(), L.Bins()
    one = (C.c_void_p * 1)(1)
    assert lib.pvg_render_bwd_views(C.byref(g), 1, C.byref(cam), C.byref(fr), C.byref(geom), C.byref(bins), one,
                                    one, one, C.byref(gg), 0, 1, 1 << 20, None) == L.PVG_ERR_INVALID
    assert "densify" in L.last_error()


def test_noalloc_bin_sort_rejects_an_oversized_plan_on_host(lib):
    """The library-held scratch has a fixed size: a bin sort whose plan needs
    more is refused before any device call (the arrays are never touched)."""
    from paper_2311_18561_amd import _lib as L
    geom = L.Geom()
    geom.n = 4_000_000
    geom.xy = geom.depth = geom.conic_op = geom.rgb = geom.radius = geom.tiles = 16
    cam = L.Camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.znear = 1920, 1280, 1500.0, 1500.0, 960.0, 640.0, 0.2
    cam.R[:] = [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0]
    bins = L.Bins()
    bins.capacity = 40_000_000
    bins.keys = bins.vals = bins.ranges = bins.counters = 16
    bins.tile_cull = 1
    assert lib.pvg_bin_sort_noalloc(C.byref(geom), C.byref(cam), C.byref(bins), 1, None) == L.PVG_ERR_NOMEM
    msg = L.last_error()
    assert "library-held scratch" in msg and str(L.NOALLOC_SCRATCH_BYTES) in msg
    ws = L.WsSizes()
    assert lib.pvg_workspace_query(geom.n, 1920, 1280, bins.capacity, C.byref(ws)) == 0
    assert ws.bin_tmp_bytes > L.NOALLOC_SCRATCH_BYTES
    bins.capacity = -1
    assert lib.pvg_bin_sort_noalloc(C.byref(geom), C.byref(cam), C.byref(bins), 1, None) == L.PVG_ERR_INVALID


def test_misaligned_workspace_refused_on_host(lib):
    """A workspace that does not start on a 256-byte boundary is refused
    before any device call, after the size check (the pointers are never
    dereferenced on the host; nothing is launched)."""
    from paper_2311_18561_amd import _lib as L
    geom = L.Geom()
    geom.n = 1000
    geom.xy = geom.depth = geom.conic_op = geom.rgb = geom.radius = geom.tiles = 256
    cam = L.Camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.znear = 64, 48, 50.0, 50.0, 32.0, 24.0, 0.2
    cam.R[:] = [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0]
    bins = L.Bins()
    bins.capacity = 10_000
    bins.keys = bins.vals = bins.ranges = bins.counters = 256
    ws = L.WsSizes()
    assert lib.pvg_workspace_query(geom.n, 64, 48, bins.capacity, C.byref(ws)) == 0
    need = int(ws.bin_tmp_bytes)
    assert lib.pvg_bin_sort(C.byref(geom), C.byref(cam), C.byref(bins), 4096 + 16, need, 0, None) == L.PVG_ERR_INVALID
    assert "256-byte boundary" in L.last_error()
    assert lib.pvg_bin_sort(C.byref(geom), C.byref(cam), C.byref(bins), 4096 + 16, need - 1, 0, None) == \
        L.PVG_ERR_NOMEM


def test_feature_entry_points_reject_bad_arguments_on_host(lib):
    """Feature compositing and its adjoint refuse a channel count outside
    [1, PVG_MAX_FEATURE_CHANNELS], a row stride below it and missing arrays
    before any device call; the scratch query grows with the channel count."""
    from paper_2311_18561_amd import _lib as L
    geom = L.Geom()
    geom.n = 10
    geom.xy = geom.depth = geom.conic_op = geom.rgb = geom.radius = geom.tiles = 16
    cam = L.Camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.znear = 64, 48, 50.0, 50.0, 32.0, 24.0, 0.2
    cam.R[:] = [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0]
    bins = L.Bins()
    bins.capacity = 100
    bins.keys = bins.vals = bins.ranges = bins.counters = 16
    for nch, ld in ((0, 4), (L.MAX_FEATURE_CHANNELS + 1, 64), (8, 7)):
        assert lib.pvg_render_features(C.byref(geom), C.byref(bins), C.byref(cam), 16, ld, nch, 16, 16, 16,
                                       None) == L.PVG_ERR_INVALID
        assert "n_ch" in L.last_error()
    assert lib.pvg_render_features(C.byref(geom), C.byref(bins), C.byref(cam), None, 4, 4, 16, 16, 16,
                                   None) == L.PVG_ERR_INVALID
    size = C.c_size_t()
    assert lib.pvg_features_bwd_tmp_bytes(10, 1, 0, 100, C.byref(size)) == L.PVG_ERR_INVALID
    assert lib.pvg_features_bwd_tmp_bytes(10, 1, L.MAX_FEATURE_CHANNELS + 1, 100, C.byref(size)) == L.PVG_ERR_INVALID
    sizes = []
    for nch in (1, 4, 5, 19, 32):
        assert lib.pvg_features_bwd_tmp_bytes(1000, 2, nch, 100_000, C.byref(size)) == 0
        sizes.append(size.value)
    assert sizes[0] == sizes[1] and sizes[1] < sizes[2] < sizes[3] < sizes[4]
    # records hold 6 + (n_ch rounded up to a kernel width) floats per instance
    assert sizes[4] - sizes[1] >= 4 * (32 - 4) * 100_000
    g = L.Gaussians()
    g.n = 10
    gg = L.GaussiansGrad()
    one = (C.c_void_p * 1)(16)
    args = (C.byref(g), 1, C.byref(cam), C.byref(L.Frame()), C.byref(geom), C.byref(bins), one, one)
    assert lib.pvg_render_features_bwd(*args, 16, 4, 0, one, 16, C.byref(gg), 0, 16, 1 << 20,
                                       None) == L.PVG_ERR_INVALID


def test_l1_loss_arguments_checked_on_host(lib):
    """pvg_l1_loss: the header's scratch size matches the binding's, and a
    negative count or a missing array is rejected before any launch."""
    import re

    from paper_2311_18561_amd import _lib as L
    hdr = open(os.path.join(ROOT, "include", "pvg.h")).read()
    assert int(re.search(r"#define PVG_L1_PARTIALS (\d+)", hdr).group(1)) == L.L1_PARTIALS
    buf = (C.c_float * 8)()
    p = C.cast(buf, C.c_void_p)
    assert lib.pvg_l1_loss(p, p, -1, 1.0, p, p, p, None) == L.PVG_ERR_INVALID
    for k in range(4):  # a, b, loss, partials
        args = [p, p, 4, 1.0, p, p, p, None]
        args[[0, 1, 4, 6][k]] = None
        assert lib.pvg_l1_loss(*args) == L.PVG_ERR_INVALID
