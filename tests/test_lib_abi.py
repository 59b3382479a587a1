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
