"""Flexible rendering channels (Sec. 3.1) on the GPU against the oracle: the
blended camera depth sum T alpha z, the rendered opacity O = sum T alpha =
1 - final_T, the velocity map sum T alpha v~ (v~ = v exp(-beta / (2 l))) and
the staticness map sum T alpha beta / l, all differentiable outputs of
pvg_render_views.

Forward: the depth channel against the oracle's FP32 compositor (and the
images, final_T and last contributors unchanged by asking for it).  Adjoint:
a loss on image, depth and opacity together against the FP64 oracle adjoint
on the FP32 discrete structure, per element within 1e-3 of max(|g*|, 1e-2
rms(g*)), the bar of the image-only adjoint.  Pixels whose skip or stop
decisions are ambiguous (the oracle's decision margin below 1: either
branch is a correct FP32 render) are compared nowhere and carry no loss."""
import numpy as np
import pytest

import gen
from helpers import FIELDS, grad_tolerance_report, oracle_grads, oracle_margin, to_device, unambiguous


def _oracle_lists(orc, scene, cam, t, d):
    """The oracle's FP32 record and lists of one view, with 0/1 weights that
    keep the pixels whose decisions (with the alpha clamp) are unambiguous."""
    pre = orc.preprocess_f32(scene, cam, t, d)
    bins = orc.bin_sort(pre, cam)
    return pre, bins, unambiguous(oracle_margin(pre, bins, cam, t, d, gradients=True))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = [
    ("tiny", lambda: gen.make_scene(60, 7, sh_degree=3), lambda: gen.yaw_camera(80, 56, 10.0, (0.2, 0.1, -0.5)),
     0.45, (0.0, 0.05)),
    ("cfg1-20k", lambda: gen.make_config(1, n=20_000)["scene"], lambda: gen.make_config(1, n=20_000)["cameras"][0],
     0.4, (0.0, 0.05)),
]


@pytest.mark.parametrize("name,mk_scene,mk_cam,t,dts", CASES)
@pytest.mark.parametrize("tile_cull", [True, False])
def test_depth_channel_forward(orc, name, mk_scene, mk_cam, t, dts, tile_cull):
    import paper_2311_18561_amd as pvg
    scene, cam = mk_scene(), mk_cam()
    params = to_device(scene)
    views = [(cam, t, d) for d in dts]
    with torch.no_grad():
        img, depth, opac, vbar, rho = pvg.pvg_render_views(params, views, tile_cull=tile_cull, channels=True)
    for k, (_, tt, d) in enumerate(views):
        ref_img = pvg.render(params, cam, tt, d, tile_cull=tile_cull)
        assert torch.equal(img[k], ref_img[0]), k  # the channel leaves the image alone
        assert torch.equal(opac[k], 1.0 - ref_img[1]), k
        pre = orc.preprocess_f32(scene, cam, tt, d)
        bins = orc.bin_sort(pre, cam)
        clear = oracle_margin(pre, bins, cam, tt, d) >= 1.0
        o_img, o_T, o_nc, o_D, o_F = orc.render_f32(pre, bins, cam, tt, d, want_depth=True, want_feat=True)
        got = depth[k].cpu().numpy()
        scale = max(1.0, float(np.abs(o_D).max()))
        err = float(np.abs(got - o_D)[clear].max()) / scale
        print(f"[{name} cull={tile_cull} view {k}] max |depth - oracle| / max depth = {err:.3g} "
              f"({int((~clear).sum())} ambiguous pixels)")
        assert err <= 1e-5
        np.testing.assert_allclose(ref_img[1].cpu().numpy()[clear], o_T[clear], atol=1e-5)
        got_f = np.concatenate([vbar[k].cpu().numpy(), rho[k].cpu().numpy()[None]])
        fscale = max(1.0, float(np.abs(o_F).max()))
        ferr = float(np.abs(got_f - o_F)[:, clear].max()) / fscale
        print(f"[{name} cull={tile_cull} view {k}] max |velocity, staticness - oracle| / max = {ferr:.3g}")
        assert ferr <= 1e-5


@pytest.mark.parametrize("name,mk_scene,mk_cam,t,dts", CASES)
@pytest.mark.parametrize("recompute", [False, True])
def test_channel_gradients_vs_fp64(orc, name, mk_scene, mk_cam, t, dts, recompute):
    """L = sum w img + sum wD depth + sum wO opacity + sum wV velocity map +
    sum wR staticness map over two views (H(t) and the flow-translated
    render), against the oracle's FP64 adjoint with dimg = w, dD = wD,
    dT = -wO and dF = (wV, wR), summed over the views.  Each element is held
    to 1e-3 of the sum of the two views' |g*| (a view's FP32 adjoint is
    accurate relative to its own gradient; where the views cancel the total
    is smaller than either term)."""
    import paper_2311_18561_amd as pvg
    scene, cam = mk_scene(), mk_cam()
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(11)
    V = len(dts)
    lists = [_oracle_lists(orc, scene, cam, t, d) for d in dts]
    keep = np.stack([k for _, _, k in lists])
    w = (rng.standard_normal((V, 3, H, W)) * keep[:, None]).astype(np.float32)
    wD = (0.05 * rng.standard_normal((V, H, W)) * keep).astype(np.float32)
    wO = (rng.standard_normal((V, H, W)) * keep).astype(np.float32)
    wV = (rng.standard_normal((V, 3, H, W)) * keep[:, None]).astype(np.float32)
    wR = (rng.standard_normal((V, H, W)) * keep).astype(np.float32)
    params = [p.requires_grad_(True) for p in to_device(scene)]
    views = [(cam, t, d) for d in dts]
    img, depth, opac, vbar, rho = pvg.pvg_render_views(params, views, recompute=recompute, channels=True)
    cu = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    loss = ((img * cu(w)).sum() + (depth * cu(wD)).sum() + (opac * cu(wO)).sum() + (vbar * cu(wV)).sum()
            + (rho * cu(wR)).sum())
    loss.backward()
    sc64 = orc.scene64(scene)
    ref = {f: np.zeros_like(sc64[f]) for f in FIELDS}
    mag = {f: np.zeros_like(sc64[f]) for f in FIELDS}  # sum over the views of |g*|
    for k, d in enumerate(dts):
        pre, bins, _ = lists[k]
        dF = np.concatenate([wV[k], wR[k][None]]).astype(np.float64)
        part, _, terms = oracle_grads(orc, sc64, cam, t, d, 0, (0.0, 0.0, 0.0), pre, bins, w[k].astype(np.float64),
                                      dD=wD[k].astype(np.float64), dT=-wO[k].astype(np.float64), dF=dF)
        for f in FIELDS:
            ref[f] += part[f]
            mag[f] += np.maximum(np.abs(part[f]), 1e-2 * terms[f])
    for f, p in zip(FIELDS, params):
        worst, l2 = grad_tolerance_report(p.grad.detach().cpu().numpy(), ref[f], rel=1e-3, magnitude=mag[f])
        print(f"[{name} recompute={recompute}] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f


def test_channels_without_image_gradient(orc):
    """Only the depth and opacity carry a loss: the image gradient is zero and
    the result equals the oracle adjoint with dimg = 0."""
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(0)
    scene, cam, t = cfg["scene"], cfg["cameras"][0], cfg["t"]
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(3)
    pre, bins, keep = _oracle_lists(orc, scene, cam, t, 0.0)
    wD = (0.05 * rng.standard_normal((1, H, W)) * keep).astype(np.float32)
    wO = (rng.standard_normal((1, H, W)) * keep).astype(np.float32)
    params = [p.requires_grad_(True) for p in to_device(scene)]
    _, depth, opac, _, _ = pvg.pvg_render_views(params, [(cam, t)], channels=True)
    ((depth * torch.from_numpy(wD).cuda()).sum() + (opac * torch.from_numpy(wO).cuda()).sum()).backward()
    ref, _, terms = oracle_grads(orc, orc.scene64(scene), cam, t, 0.0, 0, (0.0, 0.0, 0.0), pre, bins,
                                 np.zeros((3, H, W)), dD=wD[0].astype(np.float64), dT=-wO[0].astype(np.float64))
    for f, p in zip(FIELDS, params):
        worst, l2 = grad_tolerance_report(p.grad.detach().cpu().numpy(), ref[f], rel=1e-3, terms=terms[f])
        print(f"[cfg0 channels only] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f


def test_velocity_staticness_only(orc):
    """Only the velocity and staticness maps carry a loss (the sparse velocity
    term of the objective, and a staticness term): the result equals the
    oracle adjoint with only dF set, and the gradient reaches v, beta and l
    through v~ and rho as well as every parameter alpha depends on."""
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(0)
    scene, cam, t = cfg["scene"], cfg["cameras"][0], cfg["t"]
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(4)
    pre, bins, keep = _oracle_lists(orc, scene, cam, t, 0.05)
    wV = (rng.standard_normal((1, 3, H, W)) * keep).astype(np.float32)
    wR = (rng.standard_normal((1, H, W)) * keep).astype(np.float32)
    params = [p.requires_grad_(True) for p in to_device(scene)]
    _, _, _, vbar, rho = pvg.pvg_render_views(params, [(cam, t, 0.05)], channels=True)
    ((vbar * torch.from_numpy(wV).cuda()).sum() + (rho * torch.from_numpy(wR).cuda()).sum()).backward()
    ref, _, terms = oracle_grads(orc, orc.scene64(scene), cam, t, 0.05, 0, (0.0, 0.0, 0.0), pre, bins,
                                 np.zeros((3, H, W)), dF=np.concatenate([wV[0], wR[0][None]]).astype(np.float64))
    for f, p in zip(FIELDS, params):
        worst, l2 = grad_tolerance_report(p.grad.detach().cpu().numpy(), ref[f], rel=1e-3, terms=terms[f])
        print(f"[cfg0 velocity/staticness only] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f


@pytest.mark.parametrize("name,mk_scene,mk_cam,t,dts", CASES)
@pytest.mark.parametrize("recompute", [False, True])
def test_normalized_depth_vs_fp64(orc, name, mk_scene, mk_cam, t, dts, recompute):
    """Normalized depth sum T alpha z / sum T alpha (Sec. 3.1) over two views.
    Forward: against the oracle's FP64 blended depth over 1 - final_T, per
    pixel within 5e-5 relative (FP32 sums of up to a few hundred positive
    terms in numerator and denominator), 0 exactly where no Gaussian reaches.
    Adjoint: L = sum w img + sum g Dn + sum wO opacity against the FP64
    adjoint fed the quotient rule's (dD, dT); each element held to 1e-3 of
    the sum of the |g*| of every view and every source (image, the quotient's
    numerator and denominator terms, which cancel for a Gaussian at the
    pixel's mean depth, and opacity)."""
    import paper_2311_18561_amd as pvg
    scene, cam = mk_scene(), mk_cam()
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(21)
    V = len(dts)
    lists = [_oracle_lists(orc, scene, cam, t, d) for d in dts]
    keep = np.stack([k for _, _, k in lists])
    w = (rng.standard_normal((V, 3, H, W)) * keep[:, None]).astype(np.float32)
    g = (0.05 * rng.standard_normal((V, H, W)) * keep).astype(np.float32)
    wO = (rng.standard_normal((V, H, W)) * keep).astype(np.float32)
    params = [p.requires_grad_(True) for p in to_device(scene)]
    views = [(cam, t, d) for d in dts]
    img, dn, opac, _, _ = pvg.pvg_render_views(params, views, recompute=recompute, channels=True,
                                               normalized_depth=True)
    cu = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    ((img * cu(w)).sum() + (dn * cu(g)).sum() + (opac * cu(wO)).sum()).backward()
    sc64 = orc.scene64(scene)
    ref = {f: np.zeros_like(sc64[f]) for f in FIELDS}
    mag = {f: np.zeros_like(sc64[f]) for f in FIELDS}
    zero_img = np.zeros((3, H, W))
    for k, d in enumerate(dts):
        pre, bins, _ = lists[k]
        args = (sc64, cam, t, d, 0, (0.0, 0.0, 0.0), pre, bins)
        _, _, T64, D64 = orc.render_f64(*args, want_depth=True)
        want = orc.normalized_depth_f64(D64, T64)
        got = dn[k].detach().cpu().numpy().astype(np.float64)
        rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-30)
        clear = oracle_margin(pre, bins, cam, t, d) >= 1.0
        rel[~clear] = 0.0  # ambiguous decisions: either branch is correct
        empty = (T64 == 1.0) & clear
        print(f"[{name} recompute={recompute} view {k}] normalized depth: max rel err = {rel[~empty].max():.3g}, "
              f"empty pixels {int(empty.sum())}")
        assert rel[~empty].max() <= 5e-5
        assert np.all(got[empty] == 0.0)
        dD, dT = orc.normalized_depth_bwd_f64(g[k], D64, T64)
        w64, wO64 = w[k].astype(np.float64), wO[k].astype(np.float64)
        total, _ = orc.backward_f64(*args, w64, dD=dD, dT=dT - wO64)
        parts = [oracle_grads(orc, *args, w64), oracle_grads(orc, *args, zero_img, dD=dD),
                 oracle_grads(orc, *args, zero_img, dT=dT), oracle_grads(orc, *args, zero_img, dT=-wO64)]
        for f in FIELDS:
            ref[f] += total[f]
            mag[f] += sum(np.maximum(np.abs(p[f]), 1e-2 * tm[f]) for p, _, tm in parts)
    for f, p in zip(FIELDS, params):
        worst, l2 = grad_tolerance_report(p.grad.detach().cpu().numpy(), ref[f], rel=1e-3, magnitude=mag[f])
        print(f"[{name} recompute={recompute} normalized depth] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f


def test_normalized_depth_needs_channels():
    """The normalized depth is one of the channels: asking for it without
    channels=True is an error rather than a plain image render."""
    import paper_2311_18561_amd as pvg
    with pytest.raises(ValueError):
        pvg.pvg_render_views([], [], channels=False, normalized_depth=True)
