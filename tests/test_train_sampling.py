"""Host logic of the temporal-smoothing sampling (Sec. 3.4: eta is the
probability of dt = 0, otherwise dt ~ U(-delta, +delta); Sec. 4: eta = 0.5 and
a 1.5-frame span): the share of plain views approaches eta, the offsets stay
inside the span and are spread over it, every view's render time plus its dt
is the supervising frame's time, eta = 1 switches the smoothing off (the
ablation of Sec. 4.3) and eta = 0 smooths every view, and bad arguments are
refused.  Also the host-side argument checks of the optimizer and densify
bindings, which must refuse a buffer before any kernel sees it."""
import random

import pytest

from paper_2311_18561_amd.train import temporal_smoothing_views


def test_share_and_span():
    rng = random.Random(3)
    cams = ["a", "b", "c"]
    n_plain, dts = 0, []
    for _ in range(4000):
        t_frame = rng.random()
        views, times = temporal_smoothing_views(cams, t_frame, 0.1, eta=0.3, rng=rng)
        for (cam, t, dt, mode, bg), tt in zip(views, times):
            assert mode == 0 and bg == (0.0, 0.0, 0.0)
            assert tt == t_frame  # the supervising image is the training frame's
            assert t + dt == pytest.approx(t_frame, abs=1e-15)  # Eq. (12): state at t_f - dt, moved by dt
            if dt == 0.0:
                n_plain += 1
                assert t == t_frame
            else:
                dts.append(dt)
    share = n_plain / 12000
    assert abs(share - 0.3) < 0.02
    assert max(abs(d) for d in dts) <= 0.075 + 1e-12
    assert min(dts) < -0.07 and max(dts) > 0.07  # spread over the whole span
    assert abs(sum(dts) / len(dts)) < 0.003  # centred on 0


def test_eta_limits_and_errors():
    rng = random.Random(1)
    views, _ = temporal_smoothing_views(["a"] * 50, 0.2, 0.1, eta=1.0, rng=rng)
    assert all(v[2] == 0.0 and v[1] == 0.2 for v in views)  # eta = 1: smoothing off (Sec. 4.3)
    views, _ = temporal_smoothing_views(["a"] * 50, 0.2, 0.1, eta=0.0, rng=rng)
    assert all(v[2] != 0.0 for v in views)
    for kw in (dict(eta=1.5), dict(frame_dt=0.0), dict(span_frames=-1.0)):
        args = dict(cams=["a"], t_frame=0.0, frame_dt=0.1, eta=0.5)
        args.update(kw)
        with pytest.raises(ValueError):
            temporal_smoothing_views(**args)


def test_adam_refuses_non_contiguous_parameters():
    """An in-place update of a copy would leave the caller's tensor as it was:
    non-contiguous parameters are refused before any GPU work."""
    import torch

    from paper_2311_18561_amd.optim import PVGAdam
    mu = torch.zeros((4, 3)).t()  # [3, 4] view, not contiguous
    with pytest.raises(ValueError):
        PVGAdam._in_place([mu])


def test_buffer_checks_refuse_before_any_launch():
    """check_tensor guards every buffer the Adam, moment and densify bindings
    hand to a kernel: dtype, device, shape and contiguity."""
    import torch

    from paper_2311_18561_amd.render import check_tensor
    ok = torch.zeros((3, 5))
    assert check_tensor(ok, (3, 5), "cpu", "x") is ok
    with pytest.raises(TypeError):
        check_tensor(ok.half(), (3, 5), "cpu", "x")  # a half-size buffer
    with pytest.raises(TypeError):
        check_tensor(ok.numpy(), (3, 5), "cpu", "x")
    with pytest.raises(ValueError):
        check_tensor(ok, (3, 5), "meta", "x")  # another device: a host pointer into a kernel
    with pytest.raises(ValueError):
        check_tensor(ok, (3, 6), "cpu", "x")
    with pytest.raises(ValueError):
        check_tensor(torch.zeros((5, 3)).t(), (3, 5), "cpu", "x")


def test_moment_rows_and_densify_extra_are_checked():
    """PVGAdam.set_moments_rows and densify's carried rows refuse a wrong
    dtype, device or shape (here host tensors, which never reach a kernel)."""
    import torch

    from paper_2311_18561_amd.optim import PVGAdam
    opt = PVGAdam.__new__(PVGAdam)
    opt.moments = torch.zeros((2, 17 + 3, 4))  # degree 0: 20 rows
    opt.set_moments_rows(torch.ones((40, 6)))
    assert opt.moments.shape == (2, 20, 6) and float(opt.moments.sum()) == 240.0
    for bad in (torch.ones((40, 6), dtype=torch.float16), torch.ones((39, 6)), torch.ones(40),
                torch.ones((6, 40)).t()):
        with pytest.raises((TypeError, ValueError)):
            opt.set_moments_rows(bad)


def test_dense_adam_checks_before_any_launch():
    import torch

    import paper_2311_18561_amd as pvg
    with pytest.raises(ValueError):
        pvg.DenseAdam(torch.zeros((6, 3, 4, 4)))  # a host tensor
    with pytest.raises(ValueError):
        pvg.DenseAdam(torch.zeros((6, 3, 4, 4), dtype=torch.float64))
