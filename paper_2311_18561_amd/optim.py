"""Fused Adam over the Gaussians (Sec. 4: Adam with per-parameter learning
rates; the opacity reset) on the library's kernels.  Argument marshalling
only: the update runs in ``pvg_adam_step``."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from .render import FIELDS, _check_params, _p, _stream_handle, check_tensor, gaussians_struct

# order of the learning rates in pvg_adam_config
LR_KEYS = ("mu", "scale", "rot", "sh0", "shN", "opacity", "vel", "period", "tau", "beta")


def default_lrs(scene_radius: float) -> dict:
    """The paper's rates for v (1e-3), beta (0.02) and o (0.005); the others
    as in 3DGS (mean 1.6e-4 times the scene extent, scale 5e-3, rotation
    1e-3, SH 2.5e-3 and 2.5e-3 / 20 above degree 0); tau 1e-3; the cycle
    length l fixed (a scene-wide hyper-parameter in the paper)."""
    return {"mu": 1.6e-4 * float(scene_radius), "scale": 5e-3, "rot": 1e-3, "sh0": 2.5e-3, "shN": 2.5e-3 / 20,
            "opacity": 0.005, "vel": 1e-3, "period": 0.0, "tau": 1e-3, "beta": 0.02}


# the sky cube map's rate: the paper gives none; a texel is a colour, like a
# degree-0 SH coefficient, and takes that coefficient's rate
SKY_LR = 2.5e-3


class DenseAdam:
    """Adam on one dense learnable float32 tensor (the sky cube map
    [6,3,R,R] of Sec. 3.4), updated in place by ``pvg_adam_dense``; the
    moments live here."""

    def __init__(self, param, lr: float = SKY_LR, betas=(0.9, 0.999), eps=1e-15):
        self._check(param)
        self.m = torch.zeros_like(param)
        self.v = torch.zeros_like(param)
        self.lr, self.betas, self.eps, self.t = float(lr), betas, eps, 0

    @staticmethod
    def _check(param):
        if not isinstance(param, torch.Tensor) or param.dtype != torch.float32 or not param.is_cuda \
                or not param.is_contiguous():
            raise ValueError("a contiguous float32 tensor on a GPU is required")

    def step(self, param, grad=None):
        self._check(param)
        grad = param.grad if grad is None else grad
        if grad is None:
            raise ValueError("the tensor has no gradient")
        check_tensor(grad, param.shape, param.device, "the gradient")
        if self.m.shape != param.shape or self.m.device != param.device:
            raise ValueError("the moments were made for another tensor")
        self.t += 1
        L.check(L.load().pvg_adam_dense(_p(param), _p(grad), _p(self.m), _p(self.v), param.numel(), self.lr,
                                        float(self.betas[0]), float(self.betas[1]), float(self.eps), self.t,
                                        _stream_handle()))


class PVGAdam:
    """Adam state for one set of Gaussians: moments [2, 17 + 3K, N] (m then
    v, rows in the parameter order), the step count and the rates.  step()
    updates the nine parameter tensors in place from their .grad;
    reset_opacity() caps o and clears its moments; the moments travel
    through densify as its carried rows (``moments_rows()``)."""

    def __init__(self, params, lrs: dict, betas=(0.9, 0.999), eps=1e-15):
        params, n, degree = _check_params(list(params))
        rows = sum(p.numel() // max(n, 1) for p in params) if n else 17 + 3 * (degree + 1) ** 2
        self.moments = torch.zeros((2, rows, n), dtype=torch.float32, device=params[0].device)
        self.lrs = dict(lrs)
        self.betas, self.eps, self.t = betas, eps, 0

    def _cfg(self):
        c = L.AdamConfig()
        for k, key in enumerate(LR_KEYS):
            c.lr[k] = float(self.lrs[key])
        c.beta1, c.beta2, c.eps, c.step = float(self.betas[0]), float(self.betas[1]), float(self.eps), self.t
        return c

    @staticmethod
    def _in_place(params):
        """The parameters themselves (updated in place): they must be contiguous,
        or the update would land in a copy."""
        params = list(params)
        if any(not p.is_contiguous() for p in params):
            raise ValueError("parameters updated in place must be contiguous")
        return _check_params(params)

    def step(self, params, grads=None):
        params, n, degree = self._in_place(params)
        grads = [p.grad for p in params] if grads is None else list(grads)
        if len(grads) != len(params) or any(g is None for g in grads):
            raise ValueError("every parameter needs a gradient")
        for name, g, p in zip(FIELDS, grads, params):
            check_tensor(g, p.shape, p.device, f"the gradient of {name}")
        if self.moments.shape[2] != n:
            raise ValueError("the moments were sized for another Gaussian count (carry them through densify)")
        self.t += 1
        gs = gaussians_struct(params, n, degree)
        gg = L.GaussiansGrad()
        for name, t in zip(FIELDS, grads):
            setattr(gg, name, t.data_ptr())
        c = self._cfg()
        L.check(L.load().pvg_adam_step(C.byref(gs), C.byref(gg), _p(self.moments[0]), _p(self.moments[1]),
                                       C.byref(c), _stream_handle()))

    def reset_opacity(self, params, cap=0.01):
        params, n, degree = self._in_place(params)
        gs = gaussians_struct(params, n, degree)
        L.check(L.load().pvg_opacity_reset(C.byref(gs), _p(self.moments[0]), _p(self.moments[1]), float(cap),
                                           _stream_handle()))

    def moments_rows(self):
        """The moments as [2 (17 + 3K), N] rows for densify's extra rows."""
        return self.moments.reshape(-1, self.moments.shape[2])

    def set_moments_rows(self, rows):
        """Take the moments back from densify's carried rows [2 (17 + 3K), N']."""
        if not isinstance(rows, torch.Tensor) or rows.dim() != 2:
            raise ValueError("moment rows must be a 2-D tensor")
        check_tensor(rows, (self.moments.shape[0] * self.moments.shape[1], rows.shape[1]), self.moments.device,
                     "the moment rows")
        self.moments = rows.reshape(2, -1, rows.shape[1])
