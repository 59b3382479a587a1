"""PyTorch face of the PVG rasterizer: buffers and streams from torch, all
computation in libpvg's HIP kernels.

Parameter tensors use the library's SoA layout (float32, contiguous, on one
GPU): mu [3,N], scale [3,N], rot [4,N] (w,x,y,z), sh [K,3,N] with
K = (D+1)^2, opacity [N], vel [3,N], period [N], tau [N], beta [N].

``PVGRender.apply(mu, scale, rot, sh, opacity, vel, period, tau, beta, cam, t,
dt=0, advect_mode=0, bg=(0,0,0), recompute=True)`` renders Eq. (8) of the
paper (the flow-translated Eq. (12) render when dt != 0) and returns the image
[3,H,W]; its backward returns gradients for the nine parameter tensors.  With
``recompute=True`` only the parameters, final transmittance and contributor
counts are kept between forward and backward; the tile lists are rebuilt
(bit-identically) in the backward, so memory scales with the Gaussians and
pixels, not with pixels x depth.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _lib as L

FIELDS = ("mu", "scale", "rot", "sh", "opacity", "vel", "period", "tau", "beta")
_capacity_hint: dict = {}


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_params(params):
    mu = params[0]
    if not mu.is_cuda:
        raise ValueError("parameters must be on a GPU")
    n = mu.shape[1]
    shapes = {"mu": (3, n), "scale": (3, n), "rot": (4, n), "opacity": (n,), "vel": (3, n), "period": (n,),
              "tau": (n,), "beta": (n,)}
    out = []
    for name, t in zip(FIELDS, params):
        if t.dtype != torch.float32:
            raise TypeError(f"{name} must be float32")
        if t.device != mu.device:
            raise ValueError(f"{name} is on {t.device}, mu on {mu.device}")
        if name == "sh":
            if t.dim() != 3 or t.shape[1] != 3 or t.shape[2] != n or t.shape[0] not in (1, 4, 9, 16):
                raise ValueError(f"sh must be [K,3,N] with K in 1,4,9,16, got {tuple(t.shape)}")
        elif tuple(t.shape) != shapes[name]:
            raise ValueError(f"{name} must have shape {shapes[name]}, got {tuple(t.shape)}")
        out.append(t.contiguous())
    degree = int(round(math.sqrt(out[3].shape[0]))) - 1
    return out, n, degree


def gaussians_struct(params, n, degree) -> L.Gaussians:
    g = L.Gaussians()
    g.n = n
    g.sh_degree = degree
    for name, t in zip(FIELDS, params):
        setattr(g, name, t.data_ptr())
    return g


def camera_struct(cam: dict) -> L.Camera:
    c = L.Camera()
    R = [float(x) for x in torch.as_tensor(cam["R"], dtype=torch.float32).reshape(-1).tolist()]
    T = [float(x) for x in torch.as_tensor(cam["T"], dtype=torch.float32).reshape(-1).tolist()]
    c.R[:] = R
    c.T[:] = T
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.znear = float(cam.get("znear", 0.2))
    return c


def frame_struct(t, dt=0.0, advect_mode=0, bg=(0.0, 0.0, 0.0)) -> L.Frame:
    f = L.Frame()
    f.t, f.dt, f.advect_mode = float(t), float(dt), int(advect_mode)
    f.bg[:] = [float(b) for b in bg]
    return f


class Geom:
    """Per-Gaussian projected record (device tensors) and its ctypes view."""

    def __init__(self, n, device):
        self.n = n
        self.xy = torch.empty((n, 2), dtype=torch.float32, device=device)
        self.depth = torch.empty(n, dtype=torch.float32, device=device)
        self.conic_op = torch.empty((n, 4), dtype=torch.float32, device=device)
        self.rgb = torch.empty((n, 3), dtype=torch.float32, device=device)
        self.radius = torch.empty(n, dtype=torch.int32, device=device)
        self.tiles = torch.empty(n, dtype=torch.int32, device=device)  # uint32 counts

    def struct(self) -> L.Geom:
        g = L.Geom()
        g.n = self.n
        for f in ("xy", "depth", "conic_op", "rgb", "radius", "tiles"):
            setattr(g, f, getattr(self, f).data_ptr())
        return g


class Bins:
    """Sorted tile instances (device tensors) and their ctypes view."""

    def __init__(self, capacity, num_tiles, device, n=0):
        self.capacity = capacity
        self.keys = torch.empty(2 * max(capacity, 1), dtype=torch.int32, device=device)
        self.vals = torch.empty(2 * max(capacity, 1), dtype=torch.int32, device=device)
        self.ranges = torch.empty((num_tiles, 2), dtype=torch.int32, device=device)
        self.counters = torch.empty(4, dtype=torch.int32, device=device)
        self.first = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        self.num_instances = -1
        self.num_visible = -1

    def struct(self) -> L.Bins:
        b = L.Bins()
        b.capacity = self.capacity
        b.keys, b.vals = self.keys.data_ptr(), self.vals.data_ptr()
        b.ranges, b.counters = self.ranges.data_ptr(), self.counters.data_ptr()
        b.first = self.first.data_ptr()
        return b


def workspace(n, width, height, capacity) -> L.WsSizes:
    ws = L.WsSizes()
    L.check(L.load().pvg_workspace_query(n, width, height, capacity, C.byref(ws)))
    return ws


def preprocess(params, n, degree, cam: L.Camera, frame: L.Frame) -> Geom:
    geom = Geom(n, params[0].device)
    g = gaussians_struct(params, n, degree)
    gs = geom.struct()
    L.check(L.load().pvg_preprocess(C.byref(g), C.byref(cam), C.byref(frame), C.byref(gs), _stream_handle()))
    return geom


def bin_sort(geom: Geom, cam: L.Camera, capacity: int | None = None) -> Bins:
    """Instances sorted by (tile, depth, index); grows the capacity on demand."""
    dev = geom.xy.device
    key = (dev.index, int(cam.width), int(cam.height))
    cap = int(capacity if capacity is not None else _capacity_hint.get(key, max(1 << 16, 4 * geom.n)))
    cap = min(cap, 0xFFFFFFFF)
    lib = L.load()
    gs = geom.struct()
    for _ in range(3):
        ws = workspace(geom.n, cam.width, cam.height, cap)
        bins = Bins(cap, int(ws.num_tiles), dev, geom.n)
        tmp = torch.empty(max(int(ws.bin_tmp_bytes), 1), dtype=torch.uint8, device=dev)
        bs = bins.struct()
        st = lib.pvg_bin_sort(C.byref(gs), C.byref(cam), C.byref(bs), _p(tmp), int(ws.bin_tmp_bytes), 1,
                              _stream_handle())
        if st == L.PVG_ERR_CAPACITY:
            cap = min(int(bs.num_instances * 1.2) + 4096, 0xFFFFFFFF)
            continue
        L.check(st)
        bins.num_instances, bins.num_visible = int(bs.num_instances), int(bs.num_visible)
        if capacity is None:
            _capacity_hint[key] = max(cap, int(bins.num_instances * 1.2) + 4096)
        return bins
    raise RuntimeError("bin_sort did not converge on an instance capacity")


def render_fwd(geom: Geom, bins: Bins, cam: L.Camera, frame: L.Frame):
    dev = geom.xy.device
    H, W = int(cam.height), int(cam.width)
    img = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    final_T = torch.empty((H, W), dtype=torch.float32, device=dev)
    n_contrib = torch.empty((H, W), dtype=torch.int32, device=dev)
    gs, bs = geom.struct(), bins.struct()
    L.check(L.load().pvg_render_fwd(C.byref(gs), C.byref(bs), C.byref(cam), C.byref(frame), _p(img), _p(final_T),
                                    _p(n_contrib), _stream_handle()))
    return img, final_T, n_contrib


def render_bwd(params, n, degree, cam, frame, geom, bins, final_T, n_contrib, dL_dimg, grads=None, accumulate=False):
    dev = params[0].device
    if grads is None:
        grads = [torch.empty_like(p) for p in params]
    g = gaussians_struct(params, n, degree)
    gg = L.GaussiansGrad()
    for name, t in zip(FIELDS, grads):
        setattr(gg, name, t.data_ptr())
    ws = workspace(n, cam.width, cam.height, bins.capacity)
    tmp = torch.empty(max(int(ws.bwd_tmp_bytes), 1), dtype=torch.uint8, device=dev)
    gs, bs = geom.struct(), bins.struct()
    dL = dL_dimg.contiguous()
    L.check(L.load().pvg_render_bwd(C.byref(g), C.byref(cam), C.byref(frame), C.byref(gs), C.byref(bs), _p(final_T),
                                    _p(n_contrib), _p(dL), C.byref(gg), 1 if accumulate else 0, _p(tmp),
                                    int(ws.bwd_tmp_bytes), _stream_handle()))
    return grads


def render(params, cam: dict, t, dt=0.0, advect_mode=0, bg=(0.0, 0.0, 0.0)):
    """Forward only: returns (img [3,H,W], final_T [H,W], n_contrib [H,W], geom, bins)."""
    params, n, degree = _check_params(params)
    c, f = camera_struct(cam), frame_struct(t, dt, advect_mode, bg)
    geom = preprocess(params, n, degree, c, f)
    bins = bin_sort(geom, c)
    img, T, nc = render_fwd(geom, bins, c, f)
    return img, T, nc, geom, bins


class PVGRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu, scale, rot, sh, opacity, vel, period, tau, beta, cam, t, dt=0.0, advect_mode=0,
                bg=(0.0, 0.0, 0.0), recompute=True):
        params, n, degree = _check_params([mu, scale, rot, sh, opacity, vel, period, tau, beta])
        c, f = camera_struct(cam), frame_struct(t, dt, advect_mode, bg)
        geom = preprocess(params, n, degree, c, f)
        bins = bin_sort(geom, c)
        img, final_T, n_contrib = render_fwd(geom, bins, c, f)
        ctx.meta = (n, degree, c, f, recompute)
        ctx.kept = None if recompute else (geom, bins)
        ctx.save_for_backward(*params, final_T, n_contrib)
        return img

    @staticmethod
    def backward(ctx, dL_dimg):
        n, degree, c, f, recompute = ctx.meta
        saved = ctx.saved_tensors
        params, final_T, n_contrib = list(saved[:9]), saved[9], saved[10]
        if recompute:
            geom = preprocess(params, n, degree, c, f)
            bins = bin_sort(geom, c)
        else:
            geom, bins = ctx.kept
        grads = render_bwd(params, n, degree, c, f, geom, bins, final_T, n_contrib, dL_dimg)
        return (*grads, None, None, None, None, None, None)


def pvg_render(params, cam, t, dt=0.0, advect_mode=0, bg=(0.0, 0.0, 0.0), recompute=True):
    """Differentiable render of the nine parameter tensors (see module doc)."""
    return PVGRender.apply(*params, cam, t, dt, advect_mode, bg, recompute)
