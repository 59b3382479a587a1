"""Oracle of the SSIM loss term (Sec. 3.4 objective, weight lambda_r).

TEST INFRASTRUCTURE ONLY (see the package docstring).  FP64 numpy: the
structural similarity of Wang et al. per channel and pixel with an 11 x 11
Gaussian window (sigma 1.5, normalised), zero padding, C1 = 0.01^2 and
C2 = 0.03^2; the window sums use scipy's 2D convolution.  The gradient is
the adjoint of that definition with respect to x, pinned by finite
differences in ``tests/test_oracle_ssim.py``."""
from __future__ import annotations

import numpy as np
from scipy.signal import convolve2d

C1, C2 = 0.01 ** 2, 0.03 ** 2


def window():
    d = np.arange(11) - 5.0
    g = np.exp(-(d * d) / (2 * 1.5 ** 2))
    g /= g.sum()
    return np.outer(g, g)


def _filt(a):
    return convolve2d(a, window(), mode="same", boundary="fill", fillvalue=0.0)


def _stats(x, y):
    mx, my = _filt(x), _filt(y)
    sxx = _filt(x * x) - mx * mx
    syy = _filt(y * y) - my * my
    sxy = _filt(x * y) - mx * my
    A = 2 * mx * my + C1
    B = 2 * sxy + C2
    C = mx * mx + my * my + C1
    D = sxx + syy + C2
    return mx, my, A, B, C, D


def ssim_map(x, y):
    """S [C, H, W] for images x, y [C, H, W]."""
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    out = np.empty_like(x)
    for c in range(x.shape[0]):
        _, _, A, B, C, D = _stats(x[c], y[c])
        out[c] = (A * B) / (C * D)
    return out


def _partials(x, y):
    mx, my, A, B, C, D = _stats(x, y)
    S = (A * B) / (C * D)
    dmx = 2 * my * B / (C * D) - 2 * my * A / (C * D) - S * (2 * mx / C - 2 * mx / D)
    dexx = -S / D
    dexy = 2 * A / (C * D)
    return dmx, dexx, dexy


def ssim_grad(x, y, g, magnitude=False):
    """dL/dx for L = sum g S(x, y); with magnitude=True also the sum of the
    absolute terms of that sum (window weights are non-negative)."""
    x, y, g = (np.asarray(a, np.float64) for a in (x, y, g))
    dx = np.empty_like(x)
    mag = np.empty_like(x)
    for c in range(x.shape[0]):
        p1, p2, p3 = _partials(x[c], y[c])
        q1, q2, q3 = g[c] * p1, g[c] * p2, g[c] * p3
        dx[c] = _filt(q1) + 2 * x[c] * _filt(q2) + y[c] * _filt(q3)
        mag[c] = _filt(np.abs(q1)) + 2 * np.abs(x[c]) * _filt(np.abs(q2)) + np.abs(y[c]) * _filt(np.abs(q3))
    return (dx, mag) if magnitude else dx
