"""Training-loop pieces around the library (host logic only): the
temporal-smoothing sampling of Sec. 3.4 / Sec. 4.

Sec. 3.4 defines eta as the probability that dt = 0 (no estimated state);
otherwise dt is drawn from U(-delta, +delta) and the flow-translated
Gaussians H^ of Eq. (12) are rendered instead of H.  The ablation of Sec. 4.3
agrees (eta = 1 switches the smoothing off).  The discussion of the eta
ablation table in the appendix reads the other way (a larger eta as stronger
smoothing); the definition of Sec. 3.4 is taken here, and at the paper's
eta = 0.5 the two readings give the same draws in distribution.

The translated render supervises a training frame (the state queried at
t - dt, moved by v_bar dt, is compared with the image taken at t; Sec. 3.4):
the frame's time t_f is chosen first, then dt, and the view renders the state
at t_f - dt translated by dt, so that its render time plus dt is t_f."""
from __future__ import annotations

import random


def temporal_smoothing_views(cams, t_frame: float, frame_dt: float, eta: float = 0.5, span_frames: float = 1.5,
                             rng: random.Random | None = None, advect_mode: int = 0):
    """One iteration's views of the training frame at time t_frame, one per
    camera, as (cam, t, dt, advect_mode, bg): with probability eta the plain
    render (t = t_frame, dt = 0); otherwise dt ~ U(-delta, +delta) with
    delta = span_frames / 2 * frame_dt (a 1.5-frame span reaches 0.75 frames
    either side, Sec. 4) and t = t_frame - dt.  Returns the views and, per
    view, the time of the image that supervises it (t_frame)."""
    if not 0.0 <= eta <= 1.0 or frame_dt <= 0.0 or span_frames < 0.0:
        raise ValueError("eta in [0, 1], frame_dt > 0 and span_frames >= 0 are required")
    rng = rng or random.Random()
    delta = 0.5 * span_frames * frame_dt
    views, times = [], []
    for cam in cams:
        dt = 0.0
        if rng.random() >= eta:  # probability eta of dt = 0
            dt = (2.0 * rng.random() - 1.0) * delta
        views.append((cam, float(t_frame) - dt, float(dt), int(advect_mode), (0.0, 0.0, 0.0)))
        times.append(float(t_frame))
    return views, times
