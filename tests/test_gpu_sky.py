"""Sky refinement (Sec. 3.4) on the GPU against the oracle: the composite
C + (1 - O) f_sky(d) over a cube map and its adjoint into the opacity and the
cube map, with and without jittered rays; and the whole chain from the
Gaussians (image and opacity of pvg_render_views) through the composite."""
import numpy as np
import pytest

import gen
from helpers import FIELDS, grad_tolerance_report, oracle_grads, oracle_margin, to_device, unambiguous

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


DET = pytest.mark.parametrize("det", [False, True], ids=["scatter", "deterministic"])


@DET
@pytest.mark.parametrize("jitter", [False, True])
@pytest.mark.parametrize("res", [1, 7, 64, 1024])
def test_sky_composite_vs_oracle(orc, jitter, res, det):
    """The view crosses the +Z / +X face edge (fx = 156): cube sizes from 1
    and 7 (tens of pixels per texel) to 64 and 1024 (4.9 and 0.3), through
    the pixel-tile scatter and the deterministic texel-block gather."""
    import paper_2311_18561_amd as pvg
    cam = gen.yaw_camera(200, 136, 40.0, (0.0, 0.0, 0.0))
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(res)
    img = rng.random((3, H, W)).astype(np.float32)
    opac = rng.random((H, W)).astype(np.float32)
    cube = rng.random((6, 3, res, res)).astype(np.float32)
    jit = (rng.random((2, H, W)) - 0.5).astype(np.float32) if jitter else None
    g = rng.standard_normal((3, H, W)).astype(np.float32)
    t_img = torch.from_numpy(img).cuda().requires_grad_(True)
    t_op = torch.from_numpy(opac).cuda().requires_grad_(True)
    t_cube = torch.from_numpy(cube).cuda().requires_grad_(True)
    out = pvg.pvg_sky_composite(t_img, t_op, t_cube, cam, None if jit is None else torch.from_numpy(jit).cuda(),
                                deterministic=det)
    (out * torch.from_numpy(g).cuda()).sum().backward()
    ref = orc.sky_f64(img, opac, cube, cam, jit)
    err = float(np.abs(out.detach().cpu().numpy() - ref).max())
    print(f"[sky R={res} jitter={jitter}] max |out - oracle| = {err:.3g}")
    assert err <= 1e-6
    dO, dC = orc.sky_bwd_f64(g, opac, cube, cam, jit)
    assert np.array_equal(t_img.grad.cpu().numpy(), g)
    np.testing.assert_allclose(t_op.grad.cpu().numpy(), dO, rtol=1e-5, atol=1e-5)
    # the cube gradient sums many pixels' terms of either sign (float atomics,
    # any order): the tolerance scales with the sum of the terms' magnitudes,
    # which is the adjoint taken with |g| since (1 - O) and the bilinear weights
    # are non-negative
    _, dC_mag = orc.sky_bwd_f64(np.abs(g), opac, cube, cam, jit)
    worst, l2 = grad_tolerance_report(t_cube.grad.cpu().numpy(), dC, rel=1e-4, magnitude=dC_mag)
    print(f"[sky R={res} jitter={jitter}] cube grad worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
    assert worst <= 1.0


def test_sky_on_rendered_views_vs_fp64(orc):
    """L = sum w (C + (1 - O) f_sky(d)) for the image and opacity of a render
    (black background): gradients of the Gaussians against the FP64 render
    adjoint with dimg = w and dT = sum_c f_sky,c w_c (the composite's
    dL/dO = -that), and of the cube map against the sky adjoint."""
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(0)
    scene, cam, t = cfg["scene"], cfg["cameras"][0], cfg["t"]
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(9)
    cube = rng.random((6, 3, 16, 16)).astype(np.float32)
    pre = orc.preprocess_f32(scene, cam, t)
    bins = orc.bin_sort(pre, cam)
    # pixels whose skip or stop decisions are ambiguous carry no loss
    w = (rng.standard_normal((3, H, W)) * unambiguous(oracle_margin(pre, bins, cam, t, gradients=True))
         ).astype(np.float32)
    params = [p.requires_grad_(True) for p in to_device(scene)]
    t_cube = torch.from_numpy(cube).cuda().requires_grad_(True)
    img, _, opac, _, _ = pvg.pvg_render_views(params, [(cam, t)], channels=True)
    out = pvg.pvg_sky_composite(img[0], opac[0], t_cube, cam)
    (out * torch.from_numpy(w).cuda()).sum().backward()
    o_op = opac[0].detach().cpu().numpy().astype(np.float64)
    dO, dC = orc.sky_bwd_f64(w, o_op, cube, cam)
    args = (orc.scene64(scene), cam, t, 0.0, 0, (0.0, 0.0, 0.0), pre, bins)
    ref, _ = orc.backward_f64(*args, w.astype(np.float64), dT=-dO)
    # the colour and the opacity upstream gradients are two sources whose terms
    # cancel in each Gaussian's sum: the tolerance scales with the sum of the
    # magnitudes of their separate gradients
    ref_c, _, t_c = oracle_grads(orc, *args, w.astype(np.float64))
    ref_o, _, t_o = oracle_grads(orc, *args, np.zeros_like(w, np.float64), dT=-dO)
    for f, p in zip(FIELDS, params):
        mag = np.maximum(np.abs(ref_c[f]), 1e-2 * t_c[f]) + np.maximum(np.abs(ref_o[f]), 1e-2 * t_o[f])
        worst, l2 = grad_tolerance_report(p.grad.detach().cpu().numpy(), ref[f], rel=1e-3, magnitude=mag)
        print(f"[cfg0 + sky] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f
    _, dC_mag = orc.sky_bwd_f64(np.abs(w), o_op, cube, cam)
    worst, l2 = grad_tolerance_report(t_cube.grad.cpu().numpy(), dC, rel=1e-4, magnitude=dC_mag)
    print(f"[cfg0 + sky] cube: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
    assert worst <= 1.0


@DET
@pytest.mark.parametrize("yaw", [-45.0, 0.0, 45.0])
def test_sky_full_frame_bench_cameras(orc, yaw, det):
    """The benchmark's shape: 1920 x 1280 views (fx = 1500) at yaw -45, 0 and
    +45 degrees with a 1024 x 1024 cube map and jittered rays.  The yawed
    views look at the edge between two faces, so tiles take the LDS box, the
    mixed-face path and the direct atomics at the real pixel / texel ratio.
    Whole output, dL/dO and cube gradient against the oracle, with the bars
    of test_sky_composite_vs_oracle."""
    import paper_2311_18561_amd as pvg
    cam = gen.yaw_camera(1920, 1280, yaw, (0.0, 0.0, 50.0))
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(int(yaw) + 100)
    img = rng.random((3, H, W)).astype(np.float32)
    opac = rng.random((H, W)).astype(np.float32)
    cube = rng.random((6, 3, 1024, 1024)).astype(np.float32)
    jit = (rng.random((2, H, W)) - 0.5).astype(np.float32)
    g = rng.standard_normal((3, H, W)).astype(np.float32)
    t_op = torch.from_numpy(opac).cuda().requires_grad_(True)
    t_cube = torch.from_numpy(cube).cuda().requires_grad_(True)
    out = pvg.pvg_sky_composite(torch.from_numpy(img).cuda(), t_op, t_cube, cam, torch.from_numpy(jit).cuda(),
                                deterministic=det)
    (out * torch.from_numpy(g).cuda()).sum().backward()
    ref = orc.sky_f64(img, opac, cube, cam, jit)
    err = float(np.abs(out.detach().cpu().numpy() - ref).max())
    dO, dC = orc.sky_bwd_f64(g, opac, cube, cam, jit)
    _, dC_mag = orc.sky_bwd_f64(np.abs(g), opac, cube, cam, jit)
    np.testing.assert_allclose(t_op.grad.cpu().numpy(), dO, rtol=1e-5, atol=1e-5)
    worst, l2 = grad_tolerance_report(t_cube.grad.cpu().numpy(), dC, rel=1e-4, magnitude=dC_mag)
    faces = int(np.count_nonzero(np.abs(dC).reshape(6, -1).sum(axis=1)))
    print(f"[sky 1920x1280 yaw {yaw}] max |out - oracle| = {err:.3g}, cube grad worst/tol = {worst:.3g}, "
          f"faces reached {faces}")
    assert err <= 1e-6
    assert worst <= 1.0


def _sky_case(orc, cam, res, jit, seed, views=1, det=False):
    """Composite and adjoint of `views` views (all at camera `cam`, each with
    its own image, opacity, jitter and upstream gradient) over one cube map,
    through pvg_sky_composite_views, against the oracle summed over views."""
    import paper_2311_18561_amd as pvg
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(seed)
    img = rng.random((views, 3, H, W)).astype(np.float32)
    opac = rng.random((views, H, W)).astype(np.float32)
    cube = rng.random((6, 3, res, res)).astype(np.float32)
    g = rng.standard_normal((views, 3, H, W)).astype(np.float32)
    t_op = torch.from_numpy(opac).cuda().requires_grad_(True)
    t_cube = torch.from_numpy(cube).cuda().requires_grad_(True)
    t_jit = None if jit is None else torch.from_numpy(jit).cuda()
    out = pvg.pvg_sky_composite_views(torch.from_numpy(img).cuda(), t_op, t_cube, [cam] * views, t_jit,
                                      deterministic=det)
    (out * torch.from_numpy(g).cuda()).sum().backward()
    dC = np.zeros((6, 3, res, res))
    dC_mag = np.zeros_like(dC)
    for k in range(views):
        jk = None if jit is None else jit[k]
        ref = orc.sky_f64(img[k], opac[k], cube, cam, jk)
        assert float(np.abs(out[k].detach().cpu().numpy() - ref).max()) <= 1e-6
        dO, dCk = orc.sky_bwd_f64(g[k], opac[k], cube, cam, jk)
        np.testing.assert_allclose(t_op.grad[k].cpu().numpy(), dO, rtol=1e-5, atol=1e-5)
        dC += dCk
        dC_mag += orc.sky_bwd_f64(np.abs(g[k]), opac[k], cube, cam, jk)[1]
    worst, l2 = grad_tolerance_report(t_cube.grad.cpu().numpy(), dC, rel=1e-4, magnitude=dC_mag)
    return worst, l2


@DET
@pytest.mark.parametrize("res", [64, 1024])
def test_sky_jitter_beyond_half_pixel(orc, res, det):
    """Jitter up to 1.5 pixels (two thirds of the pixels beyond the half
    pixel that the gather's pixel rectangles allow for): in the deterministic
    form those pixels take the per-pixel atomic pass, the rest the gather;
    every pixel's dL/dO and every texel against the oracle."""
    cam = gen.yaw_camera(200, 136, 40.0, (0.0, 0.0, 0.0))
    rng = np.random.default_rng(res + 7)
    jit = ((rng.random((1, 2, 136, 200)) - 0.5) * 3.0).astype(np.float32)
    worst, l2 = _sky_case(orc, cam, res, jit, res + 8, det=det)
    print(f"[sky wide jitter R={res} det={det}] cube grad worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
    assert worst <= 1.0


@DET
@pytest.mark.parametrize("fx,res", [(None, 512), (150.0, 256), (150.0, 16)])
def test_sky_pitched_camera(orc, fx, res, det):
    """A camera pitched 70 degrees about x (the view centred near the +Y
    face; at fx = 150 a 130-degree field that reaches several faces and
    texel blocks partly behind the camera) at 640 x 480, three views over
    one cube, at 2, 1.2 and 19 pixels per texel."""
    import math
    a = math.radians(70.0)
    R = np.array([[1.0, 0.0, 0.0], [0.0, math.cos(a), -math.sin(a)], [0.0, math.sin(a), math.cos(a)]])
    cam = gen.make_camera(640, 480, R=R, fx=fx)
    rng = np.random.default_rng(res)
    jit = (rng.random((3, 2, 480, 640)) - 0.5).astype(np.float32)
    worst, l2 = _sky_case(orc, cam, res, jit, res + 1, views=3, det=det)
    print(f"[sky pitched fx={fx} R={res} det={det}] cube grad worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
    assert worst <= 1.0


@DET
def test_sky_full_frame_coarse_map(orc, det):
    """The benchmark's frame (1920 x 1280, fx = 1500, yaw 45) over a coarse
    128 x 128 cube map (23 pixels per texel) at full size."""
    cam = gen.yaw_camera(1920, 1280, 45.0, (0.0, 0.0, 50.0))
    rng = np.random.default_rng(128)
    jit = (rng.random((1, 2, 1280, 1920)) - 0.5).astype(np.float32)
    worst, l2 = _sky_case(orc, cam, 128, jit, 129, det=det)
    print(f"[sky 1920x1280 R=128 det={det}] cube grad worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
    assert worst <= 1.0


@DET
@pytest.mark.parametrize("scale", [1e-30, 1e30])
def test_sky_gradient_extreme_scales(orc, scale, det):
    """Upstream gradients of magnitude 1e-30 and 1e30: the fixed-point sums
    take their scale from each tile's or block's bound, so the cube gradient
    keeps its relative accuracy at both ends."""
    import paper_2311_18561_amd as pvg
    cam = gen.yaw_camera(200, 136, 40.0, (0.0, 0.0, 0.0))
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(31)
    opac = rng.random((H, W)).astype(np.float32)
    jit = (rng.random((2, H, W)) - 0.5).astype(np.float32)
    g = (rng.standard_normal((3, H, W)) * scale).astype(np.float32)
    for res in (64, 7):
        cube = rng.random((6, 3, res, res)).astype(np.float32)
        t_op = torch.from_numpy(opac).cuda().requires_grad_(True)
        t_cube = torch.from_numpy(cube).cuda().requires_grad_(True)
        out = pvg.pvg_sky_composite(torch.zeros((3, H, W), device="cuda"), t_op, t_cube, cam,
                                    torch.from_numpy(jit).cuda(), deterministic=det)
        out.backward(torch.from_numpy(g).cuda())
        dO, dC = orc.sky_bwd_f64(g, opac, cube, cam, jit)
        _, dC_mag = orc.sky_bwd_f64(np.abs(g), opac, cube, cam, jit)
        np.testing.assert_allclose(t_op.grad.cpu().numpy(), dO, rtol=1e-5, atol=1e-5 * scale)
        worst, l2 = grad_tolerance_report(t_cube.grad.cpu().numpy(), dC, rel=1e-4, magnitude=dC_mag)
        print(f"[sky scale {scale:g} R={res}] cube grad worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0


@DET
def test_sky_nonfinite_gradient_and_repeatability(orc, det):
    """A NaN and an infinity in the upstream gradient: the texels their
    pixels reach come out non-finite as in the oracle (those tiles and
    blocks sum in float) and every other texel matches it.  With finite
    inputs the deterministic form gives the same cube gradient bit for bit
    on two runs."""
    import paper_2311_18561_amd as pvg
    cam = gen.yaw_camera(200, 136, 40.0, (0.0, 0.0, 0.0))
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(37)
    opac = rng.random((H, W)).astype(np.float32)
    cube = rng.random((6, 3, 64, 64)).astype(np.float32)
    jit = (rng.random((2, H, W)) - 0.5).astype(np.float32)
    g = rng.standard_normal((3, H, W)).astype(np.float32)

    def run(gg):
        t_op = torch.from_numpy(opac).cuda().requires_grad_(True)
        t_cube = torch.from_numpy(cube).cuda().requires_grad_(True)
        out = pvg.pvg_sky_composite(torch.zeros((3, H, W), device="cuda"), t_op, t_cube, cam,
                                    torch.from_numpy(jit).cuda(), deterministic=det)
        out.backward(torch.from_numpy(gg).cuda())
        return t_op.grad.cpu().numpy(), t_cube.grad.cpu().numpy()

    if det:
        a, b = run(g)[1], run(g)[1]
        assert np.array_equal(a, b)
    gb = g.copy()
    gb[0, 40, 50] = np.nan
    gb[2, 100, 150] = np.inf
    dO_gpu, dC_gpu = run(gb)
    dO, dC = orc.sky_bwd_f64(gb, opac, cube, cam, jit)
    assert np.array_equal(np.isfinite(dC_gpu), np.isfinite(dC))
    assert np.count_nonzero(~np.isfinite(dC)) > 0
    fin = np.isfinite(dC)
    _, dC_mag = orc.sky_bwd_f64(np.where(np.isfinite(gb), np.abs(gb), 0.0), opac, cube, cam, jit)
    worst, _ = grad_tolerance_report(np.where(fin, dC_gpu, 0.0), np.where(fin, dC, 0.0), rel=1e-4,
                                     magnitude=dC_mag)
    assert worst <= 1.0
    np.testing.assert_allclose(dO_gpu[np.isfinite(dO)], dO[np.isfinite(dO)], rtol=1e-5, atol=1e-5)
    assert np.array_equal(np.isfinite(dO_gpu), np.isfinite(dO))
