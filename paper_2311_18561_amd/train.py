"""Training-loop pieces around the library (host logic only): the
temporal-smoothing sampling of Sec. 3.4 / Sec. 4.  With probability eta an
iteration renders each camera's flow-translated Gaussians H^(t + dt) of
Eq. (12) at a dt drawn uniformly from a span of frames around t (1.5 frames
in the paper), supervised by the frame nearest t + dt; otherwise the plain
H(t)."""
from __future__ import annotations

import random


def temporal_smoothing_views(cams, t: float, frame_dt: float, eta: float = 0.5, span_frames: float = 1.5,
                             rng: random.Random | None = None, advect_mode: int = 0):
    """One iteration's views: for each camera (cam, t, dt, advect_mode, bg)
    with dt = 0, or with probability eta dt ~ U[-span/2, span/2] frames
    (times frame_dt, so a 1.5-frame span reaches 0.75 frames either side).
    Returns the views and, per view, the time whose target image supervises
    it (t + dt)."""
    if not 0.0 <= eta <= 1.0 or frame_dt <= 0.0 or span_frames < 0.0:
        raise ValueError("eta in [0, 1], frame_dt > 0 and span_frames >= 0 are required")
    rng = rng or random.Random()
    views, times = [], []
    for cam in cams:
        dt = 0.0
        if rng.random() < eta:
            dt = (rng.random() - 0.5) * span_frames * frame_dt
        views.append((cam, float(t), float(dt), int(advect_mode), (0.0, 0.0, 0.0)))
        times.append(float(t) + dt)
    return views, times
