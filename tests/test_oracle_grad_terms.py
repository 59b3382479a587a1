"""Pins of the oracle's gradient-term magnitudes (the scale that an FP32
adjoint's rounding is held against): the chain rule applied to the adjoint's
own screen-space gradient reproduces its parameter gradients (the chain is
linear in them, so the per-column Jacobian the magnitude is built from is
the chain's), the magnitude bounds every gradient entry from above, and the
absolute screen-space sums bound the signed ones."""
import numpy as np

import gen
import oracle
from helpers import FIELDS


def _case():
    scene = gen.make_scene(300, 17, sh_degree=3)
    cam = gen.yaw_camera(96, 64, 8.0, (0.1, 0.0, -0.5))
    return scene, cam, 0.4, 0.05


def test_chain_of_the_adjoints_own_screen_gradient():
    oracle.build(force=False)
    scene, cam, t, dt = _case()
    sc64 = oracle.scene64(scene)
    pre = oracle.preprocess_f32(scene, cam, t, dt)
    bins = oracle.bin_sort(pre, cam)
    w = np.random.default_rng(3).standard_normal((3, cam["height"], cam["width"]))
    grads, g2d = oracle.backward_f64(sc64, cam, t, dt, 0, (0.1, 0.2, 0.3), pre, bins, w)
    again, _ = oracle.backward_f64(sc64, cam, t, dt, 0, (0.1, 0.2, 0.3), pre, bins, np.zeros_like(w), g2d_in=g2d)
    for f in FIELDS:
        np.testing.assert_allclose(again[f], grads[f], rtol=1e-12, atol=1e-15, err_msg=f)


def test_magnitude_bounds_every_entry():
    oracle.build(force=False)
    scene, cam, t, dt = _case()
    sc64 = oracle.scene64(scene)
    pre = oracle.preprocess_f32(scene, cam, t, dt)
    bins = oracle.bin_sort(pre, cam)
    w = np.random.default_rng(4).standard_normal((3, cam["height"], cam["width"]))
    grads, g2d, g2a = oracle.backward_f64(sc64, cam, t, dt, 0, (0.0, 0.0, 0.0), pre, bins, w, want_abs=True)
    assert np.all(g2a[:, :9] >= np.abs(g2d[:, :9]) * (1 - 1e-12))
    _, _, mag = oracle.backward_f64(sc64, cam, t, dt, 0, (0.0, 0.0, 0.0), pre, bins, w, want_terms=True)
    cancel = []
    for f in FIELDS:
        assert np.all(mag[f] >= np.abs(grads[f]) * (1 - 1e-12)), f
        nz = np.abs(grads[f]) > 0
        cancel.append(float(np.max(mag[f][nz] / np.abs(grads[f][nz]))))
    # with random-sign pixel weights some entries cancel by orders of magnitude
    assert max(cancel) > 10.0
    # with every weight of one sign on one channel and a single pixel, a
    # screen-space entry's absolute sum equals its magnitude
    one = np.zeros_like(w)
    one[0, 30, 40] = 1.0
    _, g1, a1 = oracle.backward_f64(sc64, cam, t, dt, 0, (0.0, 0.0, 0.0), pre, bins, one, want_abs=True)
    np.testing.assert_allclose(a1[:, 6], np.abs(g1[:, 6]), rtol=1e-12)


def test_magnitude_equals_jacobian_columns_times_abs_sums():
    """The in-oracle magnitude equals the chain applied, one screen-space entry
    at a time, to unit inputs (the Jacobian's columns), in absolute value,
    weighted by the absolute sums."""
    oracle.build(force=False)
    scene, cam, t, dt = _case()
    sc64 = oracle.scene64(scene)
    pre = oracle.preprocess_f32(scene, cam, t, dt)
    bins = oracle.bin_sort(pre, cam)
    n = scene["n"]
    w = np.random.default_rng(5).standard_normal((3, cam["height"], cam["width"]))
    _, _, g2a = oracle.backward_f64(sc64, cam, t, dt, 0, (0.0, 0.0, 0.0), pre, bins, w, want_abs=True)
    _, _, mag = oracle.backward_f64(sc64, cam, t, dt, 0, (0.0, 0.0, 0.0), pre, bins, w, want_terms=True)
    ref = {f: np.zeros_like(sc64[f]) for f in FIELDS}
    for k in range(14):
        e = np.zeros((n, 14))
        e[:, k] = 1.0
        col, _ = oracle.backward_f64(sc64, cam, t, dt, 0, (0.0, 0.0, 0.0), pre, bins, np.zeros_like(w), g2d_in=e)
        for f in FIELDS:
            ref[f] += np.abs(col[f]) * g2a[:, k]
    for f in FIELDS:
        np.testing.assert_allclose(mag[f], ref[f], rtol=1e-12, atol=1e-300, err_msg=f)
