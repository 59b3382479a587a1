"""The training pieces together on the GPU, on the 2,000-Gaussian workload:
views from the temporal-smoothing sampler render as their single renders;
three iterations of channels, sky, SSIM, the Sec. 3.4 loss terms, the
view-space statistics and Adam keep every value finite and move the
parameters; a densify pass then carries the Adam moments and Adam continues
on the new Gaussian count."""
import random

import numpy as np
import pytest

import gen
from helpers import to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_sampled_views_render_as_single_renders():
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(0)
    params = to_device(cfg["scene"])
    cams = [cfg["cameras"][0], gen.yaw_camera(128, 96, 20.0, (0.0, 0.0, 0.0))]
    views, times = pvg.temporal_smoothing_views(cams, cfg["t"], 0.05, eta=0.0, rng=random.Random(2))
    assert all(v[2] != 0.0 for v in views)
    with torch.no_grad():
        imgs = pvg.pvg_render_views(params, views, stack=True)
        for k, (cam, t, dt, mode, bg) in enumerate(views):
            ref = pvg.render(params, cam, t, dt, mode, bg)[0]
            assert torch.equal(imgs[k], ref), k


def test_training_iterations_and_densify():
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(0)
    scene = cfg["scene"]
    cam, t = cfg["cameras"][0], cfg["t"]
    H, W = cam["height"], cam["width"]
    params = [p.requires_grad_(True) for p in to_device(scene)]
    before = [p.detach().clone() for p in params]
    n = scene["n"]
    acc = torch.zeros(n, device="cuda")
    cnt = torch.zeros(n, device="cuda")
    cube = torch.full((6, 3, 16, 16), 0.5, device="cuda")
    target = torch.from_numpy(cfg["targets"][0]).cuda()
    opt = pvg.PVGAdam(params, pvg.default_lrs(10.0))
    rng = random.Random(5)
    for it in range(3):
        for p in params:
            p.grad = None
        views, _ = pvg.temporal_smoothing_views([cam], t, 0.05, eta=0.5, rng=rng)
        views = [(cam, t, 0.0)] + [v for v in views if v[2] != 0.0]
        imgs, dn, opac, vbar, rho = pvg.pvg_render_views(params, views, channels=True, normalized_depth=True,
                                                         densify_stats=(acc, cnt))
        final = pvg.pvg_sky_composite(imgs[0], opac[0], cube, cam)
        ssim = pvg.pvg_ssim(final, target).mean()
        o = opac.clamp(1e-6, 1 - 1e-6)
        loss = (0.8 * (final - target).abs().mean() + 0.2 * (1 - ssim) + 0.1 * (1.0 / dn.clamp_min(1e-3)).mean()
                - 0.05 * (o * o.log()).mean() + 0.01 * vbar.abs().mean())
        assert torch.isfinite(loss)
        loss.backward()
        for p in params:
            assert torch.isfinite(p.grad).all()
        opt.step(params)
        for p in params:
            assert torch.isfinite(p).all()
    assert int(cnt.max().item()) >= 3
    moved = [not torch.equal(p.detach(), b) for p, b in zip(params, before)]
    assert sum(moved) >= 7  # every array with a nonzero rate (l's rate is 0)
    new, rows = pvg.densify([p.detach() for p in params], acc, cnt, torch.randn((8, n), device="cuda"),
                            pvg.densify_config(10.0, grad_threshold=float(np.quantile(
                                (acc / cnt.clamp_min(1)).cpu().numpy(), 0.9))), opt.moments_rows())
    m = new[0].shape[1]
    assert m > 0
    opt.set_moments_rows(rows)
    new = [p.requires_grad_(True) for p in new]
    img = pvg.pvg_render_views(new, [(cam, t)], stack=True)
    (img - target).abs().mean().backward()
    opt.step(new)
    assert all(torch.isfinite(p).all() for p in new)
    print(f"[train] 3 iterations, densify {n} -> {m} Gaussians, one more step on the new count")
