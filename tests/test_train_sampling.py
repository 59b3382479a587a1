"""Host logic of the temporal-smoothing sampling (Sec. 3.4, eta and the
1.5-frame span of Sec. 4): the share of smoothed views approaches eta, the
offsets stay inside the span and are spread over it, eta = 0 and 1 are
exact, and bad arguments are refused."""
import random

import pytest

from paper_2311_18561_amd.train import temporal_smoothing_views


def test_share_and_span():
    rng = random.Random(3)
    cams = ["a", "b", "c"]
    n_smooth, dts = 0, []
    for _ in range(4000):
        views, times = temporal_smoothing_views(cams, 0.4, 0.1, eta=0.5, rng=rng)
        for (cam, t, dt, mode, bg), tt in zip(views, times):
            assert t == 0.4 and tt == pytest.approx(0.4 + dt) and mode == 0 and bg == (0.0, 0.0, 0.0)
            if dt != 0.0:
                n_smooth += 1
                dts.append(dt)
    share = n_smooth / 12000
    assert abs(share - 0.5) < 0.02
    assert max(abs(d) for d in dts) <= 0.075 + 1e-12
    assert min(dts) < -0.07 and max(dts) > 0.07  # spread over the whole span
    assert abs(sum(dts) / len(dts)) < 0.003  # centred on t


def test_eta_limits_and_errors():
    rng = random.Random(1)
    views, _ = temporal_smoothing_views(["a"] * 50, 0.2, 0.1, eta=0.0, rng=rng)
    assert all(v[2] == 0.0 for v in views)
    views, _ = temporal_smoothing_views(["a"] * 50, 0.2, 0.1, eta=1.0, rng=rng)
    assert all(v[2] != 0.0 for v in views)
    for kw in (dict(eta=1.5), dict(frame_dt=0.0), dict(span_frames=-1.0)):
        args = dict(cams=["a"], t=0.0, frame_dt=0.1, eta=0.5)
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
