"""Pins of the oracle's decision margin (the per-pixel flag that lets a
differently-rounded FP32 renderer resolve a skip or stop decision the other
way): builds of the FP32 image oracle whose exponential is one ulp above or
below the C library's differ from it only by rounding at almost every pixel,
and on a seeded driving-path request one pixel moves by a whole skipped or
blended pair (T c / 255) while every contributor count stays the same; that
pixel, and every pixel either build moves by more than rounding, has a margin
below 1, and few pixels do."""
import numpy as np

import gen
import oracle
from helpers import image_in_set_error, oracle_image_set, oracle_margin


def _request(i):
    """Request i of the serving test's seeded stream (scene index, camera, t, bg)."""
    rng = np.random.default_rng(7)
    res = [(160, 96), (200, 136), (320, 240)]
    for k in range(i + 1):
        w, h = res[k % 3]
        sc = int(rng.integers(0, 3))
        yaw = float(rng.uniform(-40, 40))
        center = (0.0, 0.0, float(rng.uniform(0, 20))) if sc == 1 else (0.0, 0.0, 0.0)
        cam = gen.yaw_camera(w, h, yaw if sc == 1 else 0.0, center)
        t = float(np.float32(rng.uniform(0, 1)))
        bg = (0.1 * (k % 3), 0.0, 0.2)
    return sc, cam, t, bg


def test_exp_variants_bound_the_alpha_threshold_pixels():
    oracle.build(force=False)
    scene = gen.make_scene(50_000, 41, sh_degree=3, layout="path")
    found = 0
    for i in (1, 4, 11):
        sc, cam, t, bg = _request(i)
        assert sc == 1
        refs = oracle_image_set(scene, cam, t, 0.0, 0, bg)
        assert refs.shape == (3, 3, cam["height"], cam["width"])
        r = oracle.render(scene, cam, t, 0.0, 0, bg)
        margin = oracle_margin(r["pre"], r["bins"], cam, t, 0.0, 0, bg)
        moved = np.abs(refs[1:] - refs[0][None]).max(axis=(0, 1)) > 2e-6
        assert np.all(margin[moved] < 1.0)
        assert (margin < 1.0).mean() < 1e-3
        per = np.abs(refs[1:] - refs[0][None]).max(axis=1)
        small = per <= 2e-6
        assert small.mean() > 0.9999
        big = per[~small]
        # a flipped alpha test moves a pixel by one pair's blend, at most T c / 255
        assert np.all(big <= 0.99 * 4.0 / 255.0)
        found += int((~small).sum())
        err, edge = image_in_set_error(refs[0], refs)
        assert err == 0.0 and edge == 0
    print(f"pixels moved by a one-ulp exponential: {found}")
    assert found >= 1
