"""Position-aware adaptive control (Sec. 3.3, Eq. (9)) over the library's
densify kernels: clone, split and prune driven by the view-space gradient
statistics that the adjoint accumulates (``pvg_render_views(...,
densify_stats=(accum, count))``).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from .render import FIELDS, _check_params, _p, _stream_handle, check_tensor, gaussians_struct


def densify_config(scene_radius, grad_threshold=1.7e-4, clone_scale=None, prune_scale=None, min_opacity=0.0,
                   split_scale_decay=0.8, split_beta_decay=1.0) -> L.DensifyConfig:
    """clone_scale (g) and prune_scale (b) default to 0.01 r and 0.1 r."""
    r = float(scene_radius)
    return L.DensifyConfig(float(grad_threshold), r, 0.01 * r if clone_scale is None else float(clone_scale),
                           0.1 * r if prune_scale is None else float(prune_scale), float(min_opacity),
                           float(split_scale_decay), float(split_beta_decay))


def densify(params, grad_accum, grad_count, noise, cfg: L.DensifyConfig, extra=None):
    """One pass over the nine parameter tensors (SoA [rows, N] float32 on
    the GPU): returns (new parameter tensors, new extra rows or None).
    grad_accum, grad_count: [N] statistics; noise: [8, N] standard normal
    draws for the split children; extra: optional [R, N] rows carried along
    (kept for surviving originals, zero for new Gaussians)."""
    params, n, degree = _check_params(list(params))
    dev = params[0].device
    for t, shp, what in ((grad_accum, (n,), "grad_accum"), (grad_count, (n,), "grad_count"),
                         (noise, (8, n), "noise")):
        check_tensor(t, shp, dev, what)
    if extra is not None:
        if not isinstance(extra, torch.Tensor) or extra.dim() != 2:
            raise ValueError("extra must be a [R, N] tensor")
        check_tensor(extra, (extra.shape[0], n), dev, "extra")
    lib = L.load()
    size = C.c_size_t()
    L.check(lib.pvg_densify_tmp_bytes(n, C.byref(size)))
    tmp = torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=dev)
    g = gaussians_struct(params, n, degree)
    n_out = C.c_int64()
    L.check(lib.pvg_densify_plan(C.byref(g), _p(grad_accum), _p(grad_count), _p(noise), C.byref(cfg), _p(tmp),
                                 int(tmp.numel()), C.byref(n_out), _stream_handle()))
    m = int(n_out.value)
    out = [torch.empty((*p.shape[:-1], m), dtype=torch.float32, device=dev) for p in params]
    go = gaussians_struct(out, m, degree)
    rows = 0 if extra is None else int(extra.shape[0])
    extra_out = None if extra is None else torch.empty((rows, m), dtype=torch.float32, device=dev)
    L.check(lib.pvg_densify_apply(C.byref(g), _p(noise), C.byref(cfg), _p(tmp), int(tmp.numel()), C.byref(go), rows,
                                  _p(extra), _p(extra_out), _stream_handle()))
    return out, extra_out


def split_by_staticness(params, rho_threshold):
    """Static and dynamic Gaussians (rho = beta / l >= rho_threshold is
    static, Sec. 3.2): returns (static parameter tensors, dynamic ones),
    each in index order."""
    params, n, degree = _check_params(list(params))
    dev = params[0].device
    lib = L.load()
    size = C.c_size_t()
    L.check(lib.pvg_densify_tmp_bytes(n, C.byref(size)))
    tmp = torch.empty(max(int(size.value), 1), dtype=torch.uint8, device=dev)
    g = gaussians_struct(params, n, degree)
    n_static = C.c_int64()
    L.check(lib.pvg_staticness_split_plan(C.byref(g), float(rho_threshold), _p(tmp), int(tmp.numel()),
                                          C.byref(n_static), _stream_handle()))
    ns = int(n_static.value)
    outs = [[torch.empty((*p.shape[:-1], m), dtype=torch.float32, device=dev) for p in params] for m in (ns, n - ns)]
    gs, gd = gaussians_struct(outs[0], ns, degree), gaussians_struct(outs[1], n - ns, degree)
    L.check(lib.pvg_staticness_split_apply(C.byref(g), float(rho_threshold), _p(tmp), int(tmp.numel()), C.byref(gs),
                                           C.byref(gd), _stream_handle()))
    return outs[0], outs[1]


__all__ = ["densify", "densify_config", "split_by_staticness", "FIELDS"]
