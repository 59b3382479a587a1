"""The L1 term of the training loss (pvg_l1_loss) on the GPU: the mean
absolute difference and its gradient against numpy in FP64, with exact ties
(gradient 0), sizes that are not a multiple of four and an unaligned view,
and two runs of the same inputs giving the same loss bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n", [1, 7, 4096, 1_000_003, 6 * 3 * 1280 * 1920])
def test_l1_loss_vs_fp64(n):
    import paper_2311_18561_amd as pvg
    rng = np.random.default_rng(n % 1000)
    a = rng.standard_normal(n).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    ties = rng.random(n) < 0.01
    b[ties] = a[ties]
    ta = torch.from_numpy(a).cuda().requires_grad_(True)
    tb = torch.from_numpy(b).cuda()
    loss = pvg.l1_loss(ta, tb)
    (loss * 3.0).backward()
    ref = np.abs(a.astype(np.float64) - b.astype(np.float64)).mean()
    assert abs(float(loss.detach()) - ref) <= 1e-6 * ref
    d = a - b
    want = (3.0 * np.sign(d) / n).astype(np.float32)
    got = ta.grad.cpu().numpy()
    assert np.array_equal(got == 0, d == 0)
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=0)
    again = pvg.l1_loss(ta.detach(), tb)
    assert float(again) == float(loss.detach())


def test_l1_loss_unaligned_and_shaped():
    """A [V,3,H,W] pair and a view starting one float in (the scalar path)."""
    import paper_2311_18561_amd as pvg
    g = torch.Generator(device="cuda").manual_seed(3)
    a = torch.rand((2, 3, 17, 19), device="cuda", generator=g)
    b = torch.rand((2, 3, 17, 19), device="cuda", generator=g)
    ref = (a.double() - b.double()).abs().mean().item()
    assert abs(pvg.l1_loss(a, b).item() - ref) <= 1e-6 * ref
    big = torch.rand(1001, device="cuda", generator=g)
    other = torch.rand(1001, device="cuda", generator=g)
    x, y = big[1:], other[1:]
    xr = x.clone().requires_grad_(True)
    pvg.l1_loss(xr, y).backward()
    ref = (x.double() - y.double()).abs().mean().item()
    assert abs(pvg.l1_loss(x, y).item() - ref) <= 1e-6 * ref
    assert torch.equal(xr.grad, torch.sign(x - y) / 1000)


def test_l1_loss_empty():
    """No elements: NaN, as the mean of an empty tensor is in torch, and a
    gradient of the input's (empty) shape."""
    import paper_2311_18561_amd as pvg
    a = torch.empty((0, 3), device="cuda", requires_grad=True)
    loss = pvg.l1_loss(a, torch.empty((0, 3), device="cuda"))
    assert torch.isnan(loss).item()
    loss.backward()
    assert a.grad.shape == (0, 3)
