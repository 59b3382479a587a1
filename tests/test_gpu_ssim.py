"""The SSIM loss term on the GPU against the FP64 oracle: the map and the
gradient of sum g S with respect to the render, on ragged sizes (partial
tiles, borders), smooth and noisy images, and sampled crops of a full
1920 x 1280 frame (the window reaches 5 pixels, so a crop with a 5-pixel
margin gives the oracle exact values inside it; at the image border the
crop holds the border itself).

Bars.  The map: |dS| <= 1e-5 + 24 eps32 (G*x^2 + G*y^2 + 2 |G*xy|) (1 +
|S|) / D per pixel: each window sum takes 11 row and 11 column FP32
additions and a product (24 roundings of terms of size G*x^2, ...), and the
variances subtract sums of that size before D and B divide them.  The
gradient: 1e-3 of the sum of its terms' magnitudes (the oracle's), the
floor 1e-2 of their rms."""
import numpy as np
import pytest

from helpers import grad_tolerance_report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _smooth(rng, shape):
    from scipy.ndimage import gaussian_filter
    a = rng.random(shape)
    return np.stack([gaussian_filter(c, 3.0) for c in a]).astype(np.float32)


def _map_bound(x, y, S_ref):
    from scipy.signal import convolve2d

    from oracle import ssim as os_
    b = np.empty_like(S_ref)
    for c in range(x.shape[0]):
        f = lambda a: convolve2d(a, os_.window(), mode="same")  # noqa: E731
        xx, yy, xy = f(x[c] * x[c]), f(y[c] * y[c]), f(x[c] * y[c])
        mx, my = f(x[c]), f(y[c])
        D = (xx - mx * mx) + (yy - my * my) + os_.C2
        b[c] = 1e-5 + 24 * 6e-8 * (xx + yy + 2 * np.abs(xy)) / D * (1 + np.abs(S_ref[c]))
    return b


@pytest.mark.parametrize("H,W,smooth", [(37, 53, False), (96, 128, True), (16, 16, False), (5, 7, True)])
def test_ssim_vs_fp64(orc, H, W, smooth):
    import paper_2311_18561_amd as pvg
    rng = np.random.default_rng(H * W)
    mk = (lambda: _smooth(rng, (3, H, W))) if smooth else (lambda: rng.random((3, H, W)).astype(np.float32))
    x, y = mk(), mk()
    g = rng.standard_normal((3, H, W)).astype(np.float32)
    tx = torch.from_numpy(x).cuda().requires_grad_(True)
    S = pvg.pvg_ssim(tx, torch.from_numpy(y).cuda())
    (S * torch.from_numpy(g).cuda()).sum().backward()
    S_ref = orc.ssim.ssim_map(x, y)
    err = np.abs(S.detach().cpu().numpy() - S_ref)
    bound = _map_bound(x.astype(np.float64), y.astype(np.float64), S_ref)
    print(f"[ssim {H}x{W} smooth={smooth}] max |S - oracle| = {err.max():.3g} (max err/bound {np.max(err / bound):.3g})")
    assert np.all(err <= bound)
    dx, mag = orc.ssim.ssim_grad(x, y, g, magnitude=True)
    worst, l2 = grad_tolerance_report(tx.grad.cpu().numpy(), dx, rel=1e-3, magnitude=mag)
    print(f"[ssim {H}x{W} smooth={smooth}] grad worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
    assert worst <= 1.0


def test_ssim_full_frame_sampled_crops(orc):
    """1920 x 1280, the size the training step uses: the full launch, checked
    on four 48 x 48 crops (two at corners, one on an edge, one inside)."""
    import paper_2311_18561_amd as pvg
    H, W = 1280, 1920
    rng = np.random.default_rng(77)
    x = rng.random((3, H, W)).astype(np.float32)
    y = np.clip(x + 0.1 * rng.standard_normal((3, H, W)), 0, 1).astype(np.float32)
    g = rng.standard_normal((3, H, W)).astype(np.float32)
    tx = torch.from_numpy(x).cuda().requires_grad_(True)
    S = pvg.pvg_ssim(tx, torch.from_numpy(y).cuda())
    (S * torch.from_numpy(g).cuda()).sum().backward()
    S_gpu, dx_gpu = S.detach().cpu().numpy(), tx.grad.cpu().numpy()
    m = 10  # S needs 5 pixels of context; dS/dx needs 10 (the partials' own windows)
    for (r0, c0) in [(0, 0), (H - 48, W - 48), (0, 900), (600, 1000)]:
        a0, b0 = max(r0 - m, 0), max(c0 - m, 0)
        a1, b1 = min(r0 + 48 + m, H), min(c0 + 48 + m, W)
        sl = (slice(None), slice(a0, a1), slice(b0, b1))
        S_ref = orc.ssim.ssim_map(x[sl], y[sl])
        dx, mag = orc.ssim.ssim_grad(x[sl], y[sl], g[sl], magnitude=True)
        inner = (slice(None), slice(r0 - a0, r0 - a0 + 48), slice(c0 - b0, c0 - b0 + 48))
        got = S_gpu[:, r0:r0 + 48, c0:c0 + 48]
        assert np.abs(got - S_ref[inner]).max() <= 1e-5, (r0, c0)
        worst, _ = grad_tolerance_report(dx_gpu[:, r0:r0 + 48, c0:c0 + 48], dx[inner], rel=1e-3,
                                         magnitude=mag[inner])
        print(f"[ssim 1920x1280 crop {r0},{c0}] grad worst/tol = {worst:.3g}")
        assert worst <= 1.0
