"""Host-side stream plan of the multi-view forward: every view's binning is
ordered after the preprocess that writes its record (checked for every view
and lane count up to twelve, without a GPU)."""
import importlib

import pytest


@pytest.fixture(scope="module")
def plan():
    return importlib.import_module("paper_2311_18561_amd.render")._view_plan


@pytest.mark.parametrize("lanes", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("views", list(range(1, 13)))
def test_each_binning_waits_for_its_preprocess(plan, views, lanes):
    bounds, waits = plan(views, lanes)
    assert bounds[0] == 0 and bounds[-1] == views and bounds == sorted(set(bounds))
    assert len(waits) == views
    chunk = {}
    for c in range(len(bounds) - 1):
        for k in range(bounds[c], bounds[c + 1]):
            chunk[k] = c
    assert sorted(chunk) == list(range(views))
    for k, w in enumerate(waits):
        lane = k % lanes
        if chunk[k] == 0:
            # chunk 0 runs on the caller's stream (lane 0): lane 0 is ordered after it already,
            # every other lane must wait for the event recorded after it
            assert w == (None if lane == 0 else "start"), (k, w)
        else:
            # a later chunk runs on the preprocess stream: every lane, the caller's included, waits
            assert w == chunk[k], (k, w)


def test_first_view_alone_when_views_exceed_lanes(plan):
    assert plan(6, 3)[0] == [0, 1, 3, 6]
    assert plan(3, 3)[0] == [0, 3]
    assert plan(7, 3)[0] == [0, 1, 3, 6, 7]


def test_compositing_tile_map_is_a_balanced_bijection(tmp_path):
    """The block -> tile map of the compositing launches (blend.hpp), built
    for the host: each tile exactly once for every capacity up to 40000
    tiles, and the XCDs' shares within one chunk of each other."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "tile_map_check")
    subprocess.run(["/opt/rocm/bin/hipcc", "-std=c++17", "-O1", "-I", os.path.join(root, "include"), "-I",
                    os.path.join(root, "paper_2311_18561_amd", "csrc"), "-o", exe,
                    os.path.join(root, "tests", "host", "tile_map_check.cpp")], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "tile map ok" in r.stdout
