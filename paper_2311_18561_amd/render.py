"""PyTorch face of the PVG rasterizer: buffers and streams from torch, all
computation in libpvg's HIP kernels.

Parameter tensors use the library's SoA layout (float32, contiguous, on one
GPU): mu [3,N], scale [3,N], rot [4,N] (w,x,y,z), sh [K,3,N] with
K = (D+1)^2, opacity [N], vel [3,N], period [N], tau [N], beta [N].

``PVGRender.apply(mu, scale, rot, sh, opacity, vel, period, tau, beta, cam, t,
dt=0, advect_mode=0, bg=(0,0,0), recompute=True, tile_cull=True)`` renders Eq. (8) of the
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

import numpy as np
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


def check_tensor(t, shape, device, what):
    """A buffer handed to a kernel: float32, contiguous, of `shape`, on
    `device`.  Raises (before any launch) otherwise: a host tensor would pass
    a host pointer to the kernel and another dtype a buffer of another size."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{what} must be float32, got {t.dtype}")
    if t.device != torch.device(device):
        raise ValueError(f"{what} is on {t.device}, expected {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t


def gaussians_struct(params, n, degree) -> L.Gaussians:
    g = L.Gaussians()
    g.n = n
    g.sh_degree = degree
    for name, t in zip(FIELDS, params):
        setattr(g, name, t.data_ptr())
    return g


def camera_struct(cam: dict) -> L.Camera:
    c = L.Camera()
    # numpy rather than torch for the 3x3 and 3-vector: a fifth of the host time
    R = cam["R"].cpu().numpy() if isinstance(cam["R"], torch.Tensor) else cam["R"]
    T = cam["T"].cpu().numpy() if isinstance(cam["T"], torch.Tensor) else cam["T"]
    c.R[:] = np.asarray(R, dtype=np.float32).reshape(-1).tolist()
    c.T[:] = np.asarray(T, dtype=np.float32).reshape(-1).tolist()
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

    def __init__(self, n, device, feat=False):
        self.n = n
        # [n][4] mean velocity v~ and staticness rho, for the velocity and staticness channels
        self.feat = torch.empty((n, 4), dtype=torch.float32, device=device) if feat else None
        self.xy = torch.empty((n, 2), dtype=torch.float32, device=device)
        self.depth = torch.empty(n, dtype=torch.float32, device=device)
        self.conic_op = torch.empty((n, 4), dtype=torch.float32, device=device)
        self.rgb = torch.empty((n, 3), dtype=torch.float32, device=device)
        self.radius = torch.empty(n, dtype=torch.int32, device=device)
        self.tiles = torch.empty(n, dtype=torch.int32, device=device)  # uint32 counts

    def tensors(self):
        t = (self.xy, self.depth, self.conic_op, self.rgb, self.radius, self.tiles)
        return t if self.feat is None else t + (self.feat,)

    def struct(self) -> L.Geom:
        g = L.Geom()
        g.n = self.n
        for f in ("xy", "depth", "conic_op", "rgb", "radius", "tiles"):
            setattr(g, f, getattr(self, f).data_ptr())
        g.feat = None if self.feat is None else self.feat.data_ptr()
        return g


class Bins:
    """Sorted tile instances (device tensors) and their ctypes view.

    tile_cull=True lists a Gaussian only in the tiles where it can reach
    alpha >= 1/255 (images and gradients are unchanged, the lists shorter);
    False lists every tile of its screen rectangle."""

    def __init__(self, capacity, num_tiles, device, n=0, tile_cull=True):
        self.capacity = capacity
        self.tile_cull = bool(tile_cull)
        self.keys = torch.empty(2 * max(capacity, 1), dtype=torch.int32, device=device)
        self.vals = torch.empty(2 * max(capacity, 1), dtype=torch.int32, device=device)
        self.ranges = torch.empty((num_tiles, 2), dtype=torch.int32, device=device)
        self.counters = torch.empty(4, dtype=torch.int32, device=device)
        self.first = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        self.rows = torch.empty(2 * max(capacity, 1) if tile_cull else 1, dtype=torch.int32, device=device)
        self.row_base = torch.empty(max(n, 1) if tile_cull else 1, dtype=torch.int32, device=device)
        self.num_instances = -1
        self.num_visible = -1

    def struct(self) -> L.Bins:
        b = L.Bins()
        b.capacity = self.capacity
        b.keys, b.vals = self.keys.data_ptr(), self.vals.data_ptr()
        b.ranges, b.counters = self.ranges.data_ptr(), self.counters.data_ptr()
        b.first = self.first.data_ptr()
        b.tile_cull = 1 if self.tile_cull else 0
        if self.tile_cull:
            b.rows, b.row_base = self.rows.data_ptr(), self.row_base.data_ptr()
        return b

    def tensors(self):
        return (self.keys, self.vals, self.ranges, self.counters, self.first, self.rows, self.row_base)

    def num_listed(self) -> int:
        """Instances in the sorted lists (reads the device counter: synchronises)."""
        return int(self.counters[0].item()) & 0xFFFFFFFF


def workspace(n, width, height, capacity) -> L.WsSizes:
    ws = L.WsSizes()
    L.check(L.load().pvg_workspace_query(n, width, height, capacity, C.byref(ws)))
    return ws


def preprocess(params, n, degree, cam: L.Camera, frame: L.Frame, feat: bool = False) -> Geom:
    geom = Geom(n, params[0].device, feat)
    g = gaussians_struct(params, n, degree)
    gs = geom.struct()
    L.check(L.load().pvg_preprocess(C.byref(g), C.byref(cam), C.byref(frame), C.byref(gs), _stream_handle()))
    return geom


def preprocess_views(params, n, degree, cams, frames, geoms=None) -> list:
    """preprocess for several views in one pass over the parameters: one Geom
    per view (written into `geoms` when given)."""
    dev = params[0].device
    if geoms is None:
        geoms = [Geom(n, dev) for _ in cams]
    g = gaussians_struct(params, n, degree)
    nv = len(cams)
    outs = (L.Geom * nv)(*[gm.struct() for gm in geoms])
    L.check(L.load().pvg_preprocess_views(C.byref(g), nv, (L.Camera * nv)(*cams), (L.Frame * nv)(*frames), outs,
                                          _stream_handle()))
    return geoms


def bin_sort(geom: Geom, cam: L.Camera, capacity: int | None = None, tile_cull: bool = True) -> Bins:
    """Instances sorted by (tile, depth, index); grows the capacity on demand."""
    dev = geom.xy.device
    key = (dev.index, int(cam.width), int(cam.height), bool(tile_cull))
    cap = int(capacity if capacity is not None else _capacity_hint.get(key, max(1 << 16, 4 * geom.n)))
    cap = min(cap, 0xFFFFFFFF)
    lib = L.load()
    gs = geom.struct()
    for _ in range(3):
        ws = workspace(geom.n, cam.width, cam.height, cap)
        bins = Bins(cap, int(ws.num_tiles), dev, geom.n, tile_cull)
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


def bin_sort_nosync(geom: Geom, cam: L.Camera, capacity: int, tile_cull: bool = True) -> Bins:
    """bin_sort without reading the count back: on overflow the device flag
    bins.counters[2] is set and the lists are empty (see overflowed())."""
    dev = geom.xy.device
    ws = workspace(geom.n, cam.width, cam.height, capacity)
    bins = Bins(capacity, int(ws.num_tiles), dev, geom.n, tile_cull)
    tmp = torch.empty(max(int(ws.bin_tmp_bytes), 1), dtype=torch.uint8, device=dev)
    gs, bs = geom.struct(), bins.struct()
    L.check(L.load().pvg_bin_sort(C.byref(gs), C.byref(cam), C.byref(bs), _p(tmp), int(ws.bin_tmp_bytes), 0,
                                  _stream_handle()))
    return bins


def render_fwd(geom: Geom, bins: Bins, cam: L.Camera, frame: L.Frame, out=None, depth=None, vbar=None,
               rho=None, depth_norm=False, opacity=None):
    """Composite one view; `out` (optional, contiguous [3,H,W] float32)
    receives the image, `depth` (optional, contiguous [H,W] float32) the
    blended camera depth sum T alpha z (with depth_norm the normalized depth
    sum T alpha z / sum T alpha), `vbar` ([3,H,W]) and `rho` ([H,W]) the
    velocity and staticness maps (these need a Geom with feat), `opacity`
    ([H,W]) the rendered opacity sum T alpha = 1 - final_T."""
    dev = geom.xy.device
    H, W = int(cam.height), int(cam.width)
    img = torch.empty((3, H, W), dtype=torch.float32, device=dev) if out is None else out
    final_T = torch.empty((H, W), dtype=torch.float32, device=dev)
    n_contrib = torch.empty((H, W), dtype=torch.int32, device=dev)
    gs, bs = geom.struct(), bins.struct()
    if depth is None and vbar is None and rho is None and opacity is None:
        L.check(L.load().pvg_render_fwd(C.byref(gs), C.byref(bs), C.byref(cam), C.byref(frame), _p(img),
                                        _p(final_T), _p(n_contrib), _stream_handle()))
    else:
        for t, shp in ((depth, (H, W)), (vbar, (3, H, W)), (rho, (H, W)), (opacity, (H, W))):
            assert t is None or (t.is_contiguous() and t.shape == shp and t.dtype == torch.float32)
        ch = L.Channels(_p(depth), None, None, _p(vbar), _p(rho), None, None, 1 if depth_norm else 0)
        ch.opacity = _p(opacity)
        L.check(L.load().pvg_render_fwd_channels(C.byref(gs), C.byref(bs), C.byref(cam), C.byref(frame), _p(img),
                                                 _p(final_T), _p(n_contrib), C.byref(ch), _stream_handle()))
    return img, final_T, n_contrib


def render_features(geom: Geom, bins: Bins, cam: L.Camera, feats, out=None, c0=0, width=None):
    """Composite channels c0 .. c0 + width - 1 (at most the library's channel
    limit; default all of them from c0) of feats ([n, N] float32, a
    Gaussian's vector contiguous) in one walk of the view's lists; returns
    (out [width, H, W], final_T, n_contrib)."""
    dev = geom.xy.device
    H, W = int(cam.height), int(cam.width)
    nch = int(feats.shape[1])
    width = nch - c0 if width is None else width
    if out is None:
        out = torch.empty((width, H, W), dtype=torch.float32, device=dev)
    assert feats.is_contiguous() and out.is_contiguous() and out.shape == (width, H, W)
    final_T = torch.empty((H, W), dtype=torch.float32, device=dev)
    n_contrib = torch.empty((H, W), dtype=torch.int32, device=dev)
    gs, bs = geom.struct(), bins.struct()
    L.check(L.load().pvg_render_features(C.byref(gs), C.byref(bs), C.byref(cam), feats.data_ptr() + 4 * c0, nch,
                                         width, _p(out), _p(final_T), _p(n_contrib), _stream_handle()))
    return out, final_T, n_contrib


def render_features_bwd(params, n, degree, views, feats, dL_dout, feat_grad, grads=None, accumulate=False, c0=0,
                        width=None):
    """Adjoint of render_features over views [(cam, frame, geom, bins, final_T,
    n_contrib)] with upstream gradients dL_dout[k] ([width, H, W]): adds the
    vectors' gradient into feat_grad ([n, N], columns c0 ..) and writes (or
    with accumulate adds) the parameters' gradient into grads."""
    dev = params[0].device
    if grads is None:
        grads = [torch.empty_like(p) for p in params]
    nch = int(feats.shape[1])
    width = nch - c0 if width is None else width
    V = len(views)
    cams = (L.Camera * V)(*[v[0] for v in views])
    frames = (L.Frame * V)(*[v[1] for v in views])
    geoms = (L.Geom * V)(*[v[2].struct() for v in views])
    bins = (L.Bins * V)(*[v[3].struct() for v in views])
    f_t = (C.c_void_p * V)(*[v[4].data_ptr() for v in views])
    n_c = (C.c_void_p * V)(*[v[5].data_ptr() for v in views])
    dls = [d.contiguous() for d in dL_dout]
    d_l = (C.c_void_p * V)(*[d.data_ptr() for d in dls])
    g = gaussians_struct(params, n, degree)
    gg = L.GaussiansGrad()
    for name, t in zip(FIELDS, grads):
        setattr(gg, name, t.data_ptr())
    lib = L.load()
    size = C.c_size_t()
    L.check(lib.pvg_features_bwd_tmp_bytes(n, V, width, max(v[3].capacity for v in views), C.byref(size)))
    tmp = _scratch(dev, int(size.value))
    L.check(lib.pvg_render_features_bwd(C.byref(g), V, cams, frames, geoms, bins, f_t, n_c, feats.data_ptr() + 4 * c0,
                                        nch, width, d_l, feat_grad.data_ptr() + 4 * c0, C.byref(gg),
                                        1 if accumulate else 0, _p(tmp), int(tmp.numel()), _stream_handle()))
    return grads


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


_scratch_cache: dict = {}


def _scratch(dev, nbytes):
    """Grow-only scratch of the adjoint per (device, stream): reused by every
    call in stream order, so steady-state steps allocate nothing."""
    key = (dev.index, torch.cuda.current_stream(dev).cuda_stream)
    buf = _scratch_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        _scratch_cache[key] = buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    return buf


class _BwdViewsArgs:
    """The ctypes arguments of pvg_render_bwd_views for a fixed set of views,
    views = [(cam, frame, geom, bins, final_T, n_contrib)], built once (the
    multi-view autograd node builds them in its forward, so its backward only
    adds the image gradients)."""

    def __init__(self, params, n, degree, views):
        nv = len(views)
        self.nv = nv
        self.g = gaussians_struct(params, n, degree)
        self.cams = (L.Camera * nv)(*[v[0] for v in views])
        self.frames = (L.Frame * nv)(*[v[1] for v in views])
        self.geoms = (L.Geom * nv)(*[v[2].struct() for v in views])
        self.bins = (L.Bins * nv)(*[v[3].struct() for v in views])
        self.f_t = (C.c_void_p * nv)(*[v[4].data_ptr() for v in views])
        self.n_c = (C.c_void_p * nv)(*[v[5].data_ptr() for v in views])
        size = C.c_size_t()
        L.check(L.load().pvg_bwd_views_tmp_bytes(n, nv, max(int(v[0].width) for v in views),
                                                 max(int(v[0].height) for v in views),
                                                 max(v[3].capacity for v in views), C.byref(size)))
        self.tmp_bytes = int(size.value)

    def call(self, dev, dimgs, grads, accumulate, ddepths=None, dOs=None, dvbars=None, drhos=None, depths=None,
             stats=None):
        """ddepths / dOs / dvbars / drhos (optional, per view or None):
        upstream gradients of the depth channel, the rendered opacity
        1 - final_T, the velocity map [3,H,W] and the staticness map.  depths (per view or None): the
        forward's normalized depth, given when ddepths is that map's gradient.
        stats: optional (accum, count) [N] tensors that receive the view-space
        gradient statistics of the adaptive control."""
        gg = L.GaussiansGrad()
        for name, t in zip(FIELDS, grads):
            setattr(gg, name, t.data_ptr())
        if stats is not None:
            gg.densify_grad, gg.densify_count = stats[0].data_ptr(), stats[1].data_ptr()
        lists = [list(x) if x is not None else [None] * self.nv for x in (ddepths, dOs, dvbars, drhos)]
        has = [any(x[k] is not None for x in lists) for k in range(self.nv)]
        chan = any(has)
        dimgs = list(dimgs)
        if chan:  # a view with only channel gradients still needs an image gradient (zeros)
            for k in range(self.nv):
                if dimgs[k] is None and has[k]:
                    dimgs[k] = torch.zeros((3, int(self.cams[k].height), int(self.cams[k].width)),
                                           dtype=torch.float32, device=dev)
        dls = [None if d is None else d.contiguous() for d in dimgs]
        d_l = (C.c_void_p * self.nv)(*[None if d is None else d.data_ptr() for d in dls])
        tmp = _scratch(dev, self.tmp_bytes)
        if not chan:
            L.check(L.load().pvg_render_bwd_views(C.byref(self.g), self.nv, self.cams, self.frames, self.geoms,
                                                  self.bins, self.f_t, self.n_c, d_l, C.byref(gg),
                                                  1 if accumulate else 0, _p(tmp), int(tmp.numel()),
                                                  _stream_handle()))
            return grads
        cont = [[None if d is None else d.contiguous() for d in x] for x in lists]
        dn = [None] * self.nv if depths is None else [None if d is None else d.contiguous() for d in depths]
        ch = (L.Channels * self.nv)()
        for k, (z, a, b, c, d) in enumerate(zip(dn, *cont)):
            ch[k] = L.Channels(_p(z), _p(a), None, None, None, _p(c), _p(d), 0 if z is None else 1)
            ch[k].dL_dopacity = _p(b)
        L.check(L.load().pvg_render_bwd_views_channels(C.byref(self.g), self.nv, self.cams, self.frames, self.geoms,
                                                       self.bins, self.f_t, self.n_c, d_l, ch, C.byref(gg),
                                                       1 if accumulate else 0, _p(tmp), int(tmp.numel()),
                                                       _stream_handle()))
        return grads


def render_bwd_views(params, n, degree, views, grads=None, accumulate=False, ddepths=None, dOs=None, dvbars=None,
                     drhos=None, depths=None, stats=None):
    """One adjoint call for several views of the same Gaussians:
    views = [(cam, frame, geom, bins, final_T, n_contrib, dL_dimg or None)];
    the per-Gaussian chain rule of all views is summed in registers and the
    gradient written (or added) once.  ddepths / dOs / dvbars / drhos:
    optional per-view upstream gradients of the channels (dOs: of the
    rendered opacity 1 - final_T);
    depths: per view, the forward's normalized depth when ddepths is its
    gradient (None: ddepths is the gradient of sum T alpha z)."""
    if grads is None:
        grads = [torch.empty_like(p) for p in params]
    args = _BwdViewsArgs(params, n, degree, [v[:6] for v in views])
    return args.call(params[0].device, [v[6] for v in views], grads, accumulate, ddepths, dOs, dvbars, drhos, depths,
                     stats)


def render(params, cam: dict, t, dt=0.0, advect_mode=0, bg=(0.0, 0.0, 0.0), tile_cull=True):
    """Forward only: returns (img [3,H,W], final_T [H,W], n_contrib [H,W], geom, bins)."""
    params, n, degree = _check_params(params)
    c, f = camera_struct(cam), frame_struct(t, dt, advect_mode, bg)
    geom = preprocess(params, n, degree, c, f)
    bins = bin_sort(geom, c, tile_cull=tile_cull)
    img, T, nc = render_fwd(geom, bins, c, f)
    return img, T, nc, geom, bins


class PVGRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu, scale, rot, sh, opacity, vel, period, tau, beta, cam, t, dt=0.0, advect_mode=0,
                bg=(0.0, 0.0, 0.0), recompute=True, tile_cull=True):
        params, n, degree = _check_params([mu, scale, rot, sh, opacity, vel, period, tau, beta])
        c, f = camera_struct(cam), frame_struct(t, dt, advect_mode, bg)
        geom = preprocess(params, n, degree, c, f)
        bins = bin_sort(geom, c, tile_cull=tile_cull)
        img, final_T, n_contrib = render_fwd(geom, bins, c, f)
        ctx.meta = (n, degree, c, f, recompute, tile_cull)
        ctx.kept = None if recompute else (geom, bins)
        ctx.save_for_backward(*params, final_T, n_contrib)
        return img

    @staticmethod
    def backward(ctx, dL_dimg):
        n, degree, c, f, recompute, tile_cull = ctx.meta
        saved = ctx.saved_tensors
        params, final_T, n_contrib = list(saved[:9]), saved[9], saved[10]
        if recompute:
            geom = preprocess(params, n, degree, c, f)
            bins = bin_sort(geom, c, tile_cull=tile_cull)
        else:
            geom, bins = ctx.kept
        grads = render_bwd(params, n, degree, c, f, geom, bins, final_T, n_contrib, dL_dimg)
        return (*grads, None, None, None, None, None, None, None)


KEEP_FRACTION = 0.1  # recompute="auto" keeps the views' lists while they fit this share of device memory
# the list policy the last multi-view forward took (True: rebuilt in the backward), for reports
last_recompute = None
VIEW_STREAMS = 3     # views of one call run concurrently on this many lanes: the caller's stream and side streams (default priority)
_side_streams: dict = {}


def _streams(dev):
    key = dev.index
    if key not in _side_streams:
        # VIEW_STREAMS - 1 binning lanes besides the caller's stream, and one stream for later preprocess chunks
        _side_streams[key] = [torch.cuda.Stream(device=dev) for _ in range(max(VIEW_STREAMS, 1))]
    return _side_streams[key]


def _view_plan(n_views: int, n_lanes: int):
    """Preprocess chunks and stream waits of the multi-view forward.

    Returns (bounds, waits): chunk c preprocesses views bounds[c] ..
    bounds[c + 1] - 1, chunk 0 on the caller's stream (lane 0) and the
    others in order on a further stream after it; view k is binned on lane
    k mod n_lanes after waits[k]: None (lane 0, chunk 0: already ordered),
    "start" (the caller's stream after chunk 0) or the chunk index c >= 1.
    With more views than lanes the chunks are [0], [1, n_lanes), then
    n_lanes views at a time, so the first view's binning starts after one
    view's preprocess; otherwise one chunk holds every view."""
    if n_views > n_lanes:
        bounds = sorted(set([0, 1, *range(n_lanes, n_views, n_lanes), n_views]))
    else:
        bounds = [0, n_views]
    waits = []
    for k in range(n_views):
        c = next(i for i in range(len(bounds) - 1) if bounds[i] <= k < bounds[i + 1])
        if c > 0:
            waits.append(c)
        else:
            waits.append(None if k % n_lanes == 0 else "start")
    return bounds, waits


def _record(stream):
    ev = torch.cuda.Event()
    ev.record(stream)
    return ev


def _forward_views(params, n, degree, views, tile_cull, stacked=None, depths=None, vbars=None, rhos=None,
                   depth_norm=False, opacs=None, composite=None):
    """Bin and composite view k on lane k mod VIEW_STREAMS, where lane 0 is
    the caller's stream and the others are side streams forked from it and
    joined back into it (the views' latency-bound sort and scan kernels
    overlap).  Views are preprocessed in chunks, each in one pass over the
    parameters: with at most VIEW_STREAMS views all at once on the caller's
    stream; with more, the first view on the caller's stream and the others
    (views 1 .. VIEW_STREAMS - 1, then VIEW_STREAMS at a time) on a further
    side stream while the lanes bin the earlier views.
    Each view copies its overflow flag to pinned host memory right after
    binning, so the host waits only for the last binning, not for the
    compositing, before it checks the flags and returns (the images are
    ordered before any later work on the caller's stream).  A view that
    outgrew its cached capacity is redone.  With `stacked` ([V,3,H,W],
    allocated on the caller's stream) view k's image is written into
    stacked[k]; with `depths` ([V,H,W], the same) its depth channel into
    depths[k] (the normalized depth with depth_norm), and likewise the
    velocity and staticness maps into vbars ([V,3,H,W]) and rhos ([V,H,W]),
    and the rendered opacity 1 - final_T into opacs ([V,H,W]).  With
    `composite`, view k is composited by composite(k, geom, bins, cam,
    frame) (on the view's lane) instead, which returns (None, final_T,
    n_contrib) and writes its own outputs."""
    dev = params[0].device
    main = torch.cuda.current_stream(dev)
    side = _streams(dev)
    lanes = [main, *side[:-1]]
    cams = [camera_struct(cam) for cam, *_ in views]
    frames = [frame_struct(t, dt, mode, bg) for _, t, dt, mode, bg in views]
    feat = vbars is not None or rhos is not None
    geoms = [Geom(n, dev, feat) for _ in views]  # on the caller's stream; every user is joined back into it
    nl = len(lanes)
    bounds, waits = _view_plan(len(views), nl)
    preprocess_views(params, n, degree, cams[:bounds[1]], frames[:bounds[1]], geoms[:bounds[1]])
    start, ready = _record(main), {}
    if len(bounds) > 2:
        pre = side[-1]
        pre.wait_event(start)
        with torch.cuda.stream(pre):
            for c, (a, b) in enumerate(zip(bounds[1:-1], bounds[2:]), start=1):
                preprocess_views(params, n, degree, cams[a:b], frames[a:b], geoms[a:b])
                ready[c] = _record(pre)
    flags = torch.empty(len(views), dtype=torch.int32, pin_memory=True)
    plans, outs, done, flagged = [], [], [], []
    for k, (c, f, geom) in enumerate(zip(cams, frames, geoms)):
        st = lanes[k % nl]
        if waits[k] == "start":
            st.wait_event(start)
        elif waits[k] is not None:
            st.wait_event(ready[waits[k]])
        with torch.cuda.stream(st):
            cap = _capacity_hint.get((dev.index, int(c.width), int(c.height), bool(tile_cull)))
            bins = bin_sort(geom, c, tile_cull=tile_cull) if cap is None else bin_sort_nosync(geom, c, cap, tile_cull)
            flags[k].copy_(bins.counters[2], non_blocking=True)
            fe = torch.cuda.Event()
            fe.record(st)
            out = _composite_view(k, geom, bins, c, f, stacked, depths, vbars, rhos, depth_norm, opacs, composite)
            ev = None
            if st is not main:
                ev = torch.cuda.Event()
                ev.record(st)
        plans.append([c, f, geom, bins])
        outs.append(out)
        done.append((st, ev))
        flagged.append(fe)
    for st, ev in done:
        if ev is not None:
            main.wait_event(ev)
    for (st, _), (_, _, _, bins), out in zip(done, plans, outs):
        if st is not main:  # allocated on the side stream, used later on the caller's
            for tns in (*bins.tensors(), *(out if stacked is None else out[1:])):
                if tns is not None:
                    tns.record_stream(main)
    for fe in flagged:
        fe.synchronize()
    for k, flag in enumerate(flags.tolist()):
        if flag:  # this view outgrew the cached capacity: redo it with the counting path
            c, f, geom, _ = plans[k]
            bins = bin_sort(geom, c, tile_cull=tile_cull)
            plans[k][3] = bins
            outs[k] = _composite_view(k, geom, bins, c, f, stacked, depths, vbars, rhos, depth_norm, opacs,
                                      composite)
    return plans, outs


def _composite_view(k, geom, bins, c, f, stacked, depths, vbars, rhos, depth_norm, opacs, composite):
    if composite is not None:
        return composite(k, geom, bins, c, f)
    return render_fwd(geom, bins, c, f, None if stacked is None else stacked[k],
                      None if depths is None else depths[k], None if vbars is None else vbars[k],
                      None if rhos is None else rhos[k], depth_norm, None if opacs is None else opacs[k])


def render_views(params, views, tile_cull=True):
    """Forward only, several views: returns [(img, final_T, n_contrib, geom, bins)] per view;
    views = [(cam, t) | (cam, t, dt) | (cam, t, dt, advect_mode, bg)]."""
    params, n, degree = _check_params(params)
    plans, outs = _forward_views(params, n, degree, _full_views(views), tile_cull)
    return [(img, T, nc, geom, bins) for (_, _, geom, bins), (img, T, nc) in zip(plans, outs)]


def _full_views(views):
    full = []
    for v in views:
        v = tuple(v)
        cam, t = v[0], v[1]
        dt = v[2] if len(v) > 2 else 0.0
        mode = v[3] if len(v) > 3 else 0
        bg = v[4] if len(v) > 4 else (0.0, 0.0, 0.0)
        full.append((cam, float(t), float(dt), int(mode), tuple(float(b) for b in bg)))
    return full


def _bins_bytes(b: Bins) -> int:
    return sum(t.numel() * t.element_size() for t in (b.keys, b.vals, b.ranges, b.first, b.rows, b.row_base))


class PVGRenderViews(torch.autograd.Function):
    """Several renders (cameras x times) of one set of Gaussians as one node:
    the forward launches every view without a host round trip per view (one
    overflow check at the end); the backward uses each view's lists (kept
    from the forward, or rebuilt bit for bit when recompute is set: memory
    then stays O(N + pixels + one view's instances)) and adds all views'
    gradients in the kernels into one zeroed set.  recompute="auto" keeps
    the lists when they fit KEEP_FRACTION of the device memory."""

    @staticmethod
    def forward(ctx, views, recompute, tile_cull, stack, channels, stats, *tensors):
        params, n, degree = _check_params(list(tensors))
        dev = params[0].device
        stacked = depths = vbars = rhos = opacs = None
        if stack:
            V, H, W = len(views), int(views[0][0]["height"]), int(views[0][0]["width"])
            stacked = torch.empty((V, 3, H, W), dtype=torch.float32, device=dev)
            if channels:
                depths = torch.empty((V, H, W), dtype=torch.float32, device=dev)
                vbars = torch.empty((V, 3, H, W), dtype=torch.float32, device=dev)
                rhos = torch.empty((V, H, W), dtype=torch.float32, device=dev)
                opacs = torch.empty((V, H, W), dtype=torch.float32, device=dev)
        norm = channels == 2
        plans, outs = _forward_views(params, n, degree, views, tile_cull, stacked, depths, vbars, rhos, norm, opacs)
        if recompute == "auto":
            kept_bytes = sum(_bins_bytes(b) for _, _, _, b in plans)
            recompute = kept_bytes > KEEP_FRACTION * torch.cuda.get_device_properties(dev).total_memory
        global last_recompute
        last_recompute = bool(recompute)
        ctx.meta = (n, degree, bool(recompute), tile_cull, [(c, f, b.capacity) for c, f, _, b in plans])
        ctx.kept = None if recompute else [(g, b) for _, _, g, b in plans]
        ctx.bwd = None if recompute else _BwdViewsArgs(
            params, n, degree, [(c, f, g, b, T, nc) for (c, f, g, b), (_, T, nc) in zip(plans, outs)])
        saved = list(params)
        for _, T, nc in outs:
            saved += [T, nc]
        if norm:  # the quotient's adjoint reads the normalized depth back
            saved.append(depths)
        ctx.save_for_backward(*saved)
        ctx.stack = stack
        ctx.channels = channels
        ctx.stats = stats
        if channels:  # images, depth, opacity, velocity and staticness maps, each stacked over the views
            return stacked, depths, opacs, vbars, rhos
        if stack:
            return stacked
        return tuple(img for img, _, _ in outs)

    @staticmethod
    def backward(ctx, *dimgs):
        n, degree, recompute, tile_cull, plan = ctx.meta
        ddepths = dOs = dvbars = drhos = None
        if ctx.channels:
            ddepths, dOs, dvbars, drhos = ([None if d is None else d[k] for k in range(len(plan))]
                                           for d in dimgs[1:5])
        if ctx.stack:
            d = dimgs[0]
            dimgs = tuple(None if d is None else d[k] for k in range(len(plan)))
        saved = ctx.saved_tensors
        params = list(saved[:9])
        grads = [torch.empty_like(p) for p in params]
        dn = saved[9 + 2 * len(plan)] if ctx.channels == 2 else None
        if recompute:
            # one view at a time, so only one view's lists exist at once; the
            # same inputs give the forward's lists bit for bit, within its capacity
            first = True
            for k, (c, f, cap) in enumerate(plan):
                chk = [None if x is None else x[k] for x in (ddepths, dOs, dvbars, drhos)]
                if dimgs[k] is None and all(x is None for x in chk):
                    continue
                geom = preprocess(params, n, degree, c, f, feat=bool(ctx.channels))
                bins = bin_sort_nosync(geom, c, cap, tile_cull)
                render_bwd_views(params, n, degree, [(c, f, geom, bins, saved[9 + 2 * k], saved[10 + 2 * k],
                                                      dimgs[k])], grads=grads, accumulate=not first,
                                 ddepths=[chk[0]], dOs=[chk[1]], dvbars=[chk[2]], drhos=[chk[3]],
                                 depths=None if dn is None else [dn[k]], stats=ctx.stats)
                first = False
            if first:
                for gr in grads:
                    gr.zero_()
        else:  # the kept lists, final_T and n_contrib, with the arguments built in the forward
            ctx.bwd.call(params[0].device, dimgs, grads, accumulate=False, ddepths=ddepths, dOs=dOs, dvbars=dvbars,
                         drhos=drhos, depths=None if dn is None else [dn[k] for k in range(len(plan))],
                         stats=ctx.stats)
        return (None, None, None, None, None, None, *grads)


def pvg_render_views(params, views, recompute="auto", tile_cull=True, stack=False, channels=False,
                     normalized_depth=False, densify_stats=None):
    """Differentiable renders of the nine parameter tensors for several views:
    views = [(cam, t), (cam, t, dt), ... or (cam, t, dt, advect_mode, bg)];
    returns one image [3,H,W] per view, or with stack=True (views of one
    resolution) a single [V,3,H,W] tensor.  recompute: True, False or "auto"
    (see PVGRenderViews).  channels=True (implies stack) also renders the
    flexible-rendering channels of Sec. 3.1 and returns (images [V,3,H,W],
    depth [V,H,W] = sum T alpha z, opacity [V,H,W] = sum T alpha = 1 -
    final_T, velocity map [V,3,H,W] = sum T alpha v~ with v~ = v exp(-beta /
    (2 l)), staticness map [V,H,W] = sum T alpha beta / l), all
    differentiable.  normalized_depth=True (with channels) returns the
    normalized depth sum T alpha z / sum T alpha of Sec. 3.1 in place of the
    depth (0 where no Gaussian reaches the pixel).  densify_stats: optional
    (accum, count), contiguous float32 [N] tensors on the parameters' device,
    to which the backward adds, per view in which a Gaussian is visible, the
    norm of its view-space (NDC) mean gradient and 1 (the statistics of the
    adaptive control, Sec. 3.3)."""
    full = _full_views(views)
    stack = bool(stack or channels)
    if stack and len({(int(v[0]["width"]), int(v[0]["height"])) for v in full}) != 1:
        raise ValueError("stack=True needs views of one resolution")
    if normalized_depth and not channels:
        raise ValueError("normalized_depth needs channels=True")
    mode = (2 if normalized_depth else 1) if channels else 0
    if densify_stats is not None:
        n = params[0].shape[1]
        for t in densify_stats:
            if t.shape != (n,) or t.dtype != torch.float32 or not t.is_contiguous() or t.device != params[0].device:
                raise ValueError("densify_stats must be two contiguous float32 [N] tensors on the parameters' device")
        densify_stats = tuple(densify_stats)
    out = PVGRenderViews.apply(full, recompute, tile_cull, stack, mode, densify_stats, *params)
    return out


def pvg_render(params, cam, t, dt=0.0, advect_mode=0, bg=(0.0, 0.0, 0.0), recompute=True, tile_cull=True):
    """Differentiable render of the nine parameter tensors (see module doc)."""
    return PVGRender.apply(*params, cam, t, dt, advect_mode, bg, recompute, tile_cull)


class PVGSkyComposite(torch.autograd.Function):
    """Sky refinement (Sec. 3.4): C_f = C + (1 - O) f_sky(d) over a learnable
    cube map, one view: img [3,H,W] (rendered on a black background), opacity
    [H,W], cube [6,3,R,R]; the adjoint reaches img, opacity and the cube map
    (deterministic: the cube gradient's run-to-run identical form)."""

    @staticmethod
    def forward(ctx, img, opacity, cube, cam, jitter, deterministic=False):
        c = camera_struct(cam)
        H, W = int(c.height), int(c.width)
        img, opacity, cube = img.contiguous(), opacity.contiguous(), cube.contiguous()
        if img.shape != (3, H, W) or opacity.shape != (H, W) or cube.dim() != 4 or cube.shape[:2] != (6, 3) \
                or cube.shape[2] != cube.shape[3]:
            raise ValueError("pvg_sky_composite needs img [3,H,W], opacity [H,W] and cube [6,3,R,R]")
        for t in (img, opacity, cube):
            if t.dtype != torch.float32 or not t.is_cuda:
                raise ValueError("pvg_sky_composite takes float32 CUDA tensors")
        if jitter is not None:
            jitter = jitter.contiguous()
            if jitter.shape != (2, H, W) or jitter.dtype != torch.float32:
                raise ValueError("jitter must be float32 [2,H,W]")
        out = torch.empty_like(img)
        L.check(L.load().pvg_sky_composite(C.byref(c), _p(img), _p(opacity), _p(cube), int(cube.shape[-1]),
                                           _p(jitter), _p(out), _stream_handle()))
        ctx.c = c
        ctx.save_for_backward(opacity, cube, jitter if jitter is not None else torch.empty(0, device=img.device))
        ctx.has_jitter = jitter is not None
        ctx.deterministic = bool(deterministic)
        return out

    @staticmethod
    def backward(ctx, g):
        opacity, cube, jitter = ctx.saved_tensors
        g = g.contiguous()
        d_op = torch.empty_like(opacity)
        d_cube = torch.zeros_like(cube)
        lib = L.load()
        fn = lib.pvg_sky_composite_bwd_deterministic if ctx.deterministic else lib.pvg_sky_composite_bwd
        L.check(fn(C.byref(ctx.c), _p(g), _p(opacity), _p(cube), int(cube.shape[-1]),
                   _p(jitter) if ctx.has_jitter else None, _p(d_op), _p(d_cube), _stream_handle()))
        return g, d_op, d_cube, None, None, None


def pvg_sky_composite(img, opacity, cube, cam: dict, jitter=None, deterministic=False):
    """C + (1 - O) f_sky(d) for one view (see PVGSkyComposite); jitter
    (optional [2,H,W], pixels) moves each ray inside its pixel."""
    return PVGSkyComposite.apply(img, opacity, cube, cam, jitter, deterministic)


class PVGSkyCompositeViews(torch.autograd.Function):
    """The sky composite of V views of one size over one cube map: imgs
    [V,3,H,W], opacities [V,H,W], jitter [V,2,H,W] or None.  The backward
    adds every view's cube-map gradient into one array, so a step pays one
    zero fill of the cube's gradient instead of one per view plus V - 1
    sums of full-size arrays."""

    @staticmethod
    def forward(ctx, imgs, opacities, cube, cams, jitter, deterministic=False):
        cs = [camera_struct(c) for c in cams]
        V = len(cs)
        imgs, opacities, cube = imgs.contiguous(), opacities.contiguous(), cube.contiguous()
        if V == 0 or any((c.width, c.height) != (cs[0].width, cs[0].height) for c in cs):
            raise ValueError("pvg_sky_composite_views needs one or more views of one size")
        H, W = int(cs[0].height), int(cs[0].width)
        if imgs.shape != (V, 3, H, W) or opacities.shape != (V, H, W) or cube.dim() != 4 \
                or cube.shape[:2] != (6, 3) or cube.shape[2] != cube.shape[3]:
            raise ValueError("pvg_sky_composite_views needs imgs [V,3,H,W], opacities [V,H,W] and cube [6,3,R,R]")
        for t in (imgs, opacities, cube):
            if t.dtype != torch.float32 or not t.is_cuda:
                raise ValueError("pvg_sky_composite_views takes float32 CUDA tensors")
        if jitter is not None:
            jitter = jitter.contiguous()
            if jitter.shape != (V, 2, H, W) or jitter.dtype != torch.float32:
                raise ValueError("jitter must be float32 [V,2,H,W]")
        out = torch.empty_like(imgs)
        lib, st, res = L.load(), _stream_handle(), int(cube.shape[-1])
        for k in range(V):
            L.check(lib.pvg_sky_composite(C.byref(cs[k]), _p(imgs[k]), _p(opacities[k]), _p(cube), res,
                                          None if jitter is None else _p(jitter[k]), _p(out[k]), st))
        ctx.cs = cs
        ctx.save_for_backward(opacities, cube, jitter if jitter is not None else torch.empty(0, device=imgs.device))
        ctx.has_jitter = jitter is not None
        ctx.deterministic = bool(deterministic)
        return out

    @staticmethod
    def backward(ctx, g):
        opacities, cube, jitter = ctx.saved_tensors
        g = g.contiguous()
        d_op = torch.empty_like(opacities)
        d_cube = torch.zeros_like(cube)
        lib, st, res = L.load(), _stream_handle(), int(cube.shape[-1])
        fn = lib.pvg_sky_composite_bwd_deterministic if ctx.deterministic else lib.pvg_sky_composite_bwd
        for k, c in enumerate(ctx.cs):
            L.check(fn(C.byref(c), _p(g[k]), _p(opacities[k]), _p(cube), res,
                       _p(jitter[k]) if ctx.has_jitter else None, _p(d_op[k]), _p(d_cube), st))
        return g, d_op, d_cube, None, None, None


def pvg_sky_composite_views(imgs, opacities, cube, cams, jitter=None, deterministic=False):
    """C + (1 - O) f_sky(d) for V views of one size (see PVGSkyCompositeViews)."""
    return PVGSkyCompositeViews.apply(imgs, opacities, cube, list(cams), jitter, deterministic)


class PVGL1Loss(torch.autograd.Function):
    """mean |a - b| over all elements of two float32 CUDA tensors of one
    shape (the L1 term of the training loss), differentiable in a: one
    library pass (pvg_l1_loss) forms the sum and the gradient sign(a - b) / n
    together, and the backward scales that gradient by the upstream value."""

    @staticmethod
    def forward(ctx, a, b):
        if a.shape != b.shape:
            raise ValueError(f"l1_loss needs tensors of one shape, got {tuple(a.shape)} and {tuple(b.shape)}")
        for t in (a, b):
            if t.dtype != torch.float32 or not t.is_cuda or t.device != a.device:
                raise ValueError("l1_loss takes float32 CUDA tensors on one device")
        a, b = a.contiguous(), b.contiguous()
        n = a.numel()
        if n == 0:  # the mean of nothing, as torch has it
            ctx.save_for_backward(torch.zeros_like(a))
            return torch.full((), float("nan"), dtype=torch.float32, device=a.device)
        loss = torch.empty((), dtype=torch.float32, device=a.device)
        grad = torch.empty_like(a) if ctx.needs_input_grad[0] else None
        partials = torch.empty(L.L1_PARTIALS, dtype=torch.float32, device=a.device)
        L.check(L.load().pvg_l1_loss(_p(a), _p(b), n, 1.0 / max(n, 1), _p(loss), _p(grad), _p(partials),
                                     _stream_handle()))
        if grad is not None:
            ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, g):
        if not ctx.saved_tensors:  # only b asked for a gradient, which this loss does not give
            return None, None
        (grad,) = ctx.saved_tensors
        return grad * g, None


def l1_loss(a, b):
    """mean |a - b| (see PVGL1Loss)."""
    return PVGL1Loss.apply(a, b)


class PVGSSIM(torch.autograd.Function):
    """The SSIM map of a render x against a target y (both [C,H,W] float32
    on the GPU; 11 x 11 Gaussian window, sigma 1.5): the forward keeps the
    kernel's partials, the backward returns dL/dx (the target takes none)."""

    @staticmethod
    def forward(ctx, x, y):
        x, y = x.contiguous(), y.contiguous()
        if x.shape != y.shape or x.dim() != 3 or x.dtype != torch.float32 or y.dtype != torch.float32:
            raise ValueError("x and y must be float32 [C,H,W] of one shape")
        C_, H, W = (int(v) for v in x.shape)
        smap = torch.empty_like(x)
        part = torch.empty((3, C_, H, W), dtype=torch.float32, device=x.device)
        L.check(L.load().pvg_ssim_fwd(_p(x), _p(y), C_, H, W, _p(smap), _p(part), _stream_handle()))
        ctx.save_for_backward(x, y, part)
        return smap

    @staticmethod
    def backward(ctx, g):
        x, y, part = ctx.saved_tensors
        g = g.contiguous()
        dx = torch.empty_like(x)
        C_, H, W = (int(v) for v in x.shape)
        L.check(L.load().pvg_ssim_bwd(_p(g), _p(x), _p(y), _p(part), C_, H, W, _p(dx), _stream_handle()))
        return dx, None


def pvg_ssim(x, y):
    """Differentiable SSIM map of x against y (see PVGSSIM); the loss term of
    Sec. 3.4 is lambda_r (1 - mean)."""
    return PVGSSIM.apply(x, y)


class PVGRenderSemantic(torch.autograd.Function):
    """Per-Gaussian vectors (e.g. the 19 semantic class scores of Sec. 4.1)
    composited like the colour (no background), differentiable in the
    vectors and, through alpha, in the Gaussians.  Each view's lists are
    walked once for all channels (pvg_render_features); vectors wider than
    the library's channel limit go in column groups, whose adjoints add up
    (the adjoint is linear in the upstream gradient)."""

    @staticmethod
    def forward(ctx, views, feats, *tensors):
        params, n, degree = _check_params(list(tensors))
        dev = params[0].device
        if feats.dim() != 2 or feats.shape[0] != n or feats.dtype != torch.float32 or feats.device != dev:
            raise ValueError("feats must be float32 [n, N_channels] on the parameters' device")
        nch = int(feats.shape[1])
        if nch < 1:
            raise ValueError("feats needs at least one channel")
        V = len(views)
        H, W = int(views[0][0]["height"]), int(views[0][0]["width"])
        out = torch.empty((V, nch, H, W), dtype=torch.float32, device=dev)
        groups = _feature_groups(nch)

        def composite(k, geom, bins, c, f):
            for c0, w in groups:
                _, T, nc = render_features(geom, bins, c, feats, out[k, c0:c0 + w], c0, w)
            return None, T, nc

        plans, outs = _forward_views(params, n, degree, views, tile_cull=True, composite=composite)
        ctx.plans, ctx.n, ctx.degree, ctx.nch = plans, n, degree, nch
        ctx.save_for_backward(*params, feats, *[T for _, T, _ in outs], *[nc for _, _, nc in outs])
        return out

    @staticmethod
    def backward(ctx, dout):
        saved = ctx.saved_tensors
        params, feats = list(saved[:9]), saved[9]
        V = len(ctx.plans)
        Ts, ncs = saved[10:10 + V], saved[10 + V:10 + 2 * V]
        n, degree, nch = ctx.n, ctx.degree, ctx.nch
        dev = params[0].device
        grads = [torch.empty_like(p) for p in params]
        dfeat = torch.zeros((n, nch), dtype=torch.float32, device=dev)
        if dout is None:
            for gr in grads:
                gr.zero_()
            return (None, dfeat, *grads)
        dout = dout.contiguous()
        views = [(c, f, geom, bins, T, nc) for (c, f, geom, bins), T, nc in zip(ctx.plans, Ts, ncs)]
        for j, (c0, w) in enumerate(_feature_groups(nch)):
            render_features_bwd(params, n, degree, views, feats, [dout[k, c0:c0 + w] for k in range(V)], dfeat, grads,
                                accumulate=j > 0, c0=c0, width=w)
        return (None, dfeat, *grads)


def _feature_groups(nch):
    """Column groups (first channel, width) of at most the library's channel limit."""
    step = L.MAX_FEATURE_CHANNELS
    return [(c0, min(step, nch - c0)) for c0 in range(0, nch, step)]


def pvg_render_semantic(params, views, feats):
    """Composited per-Gaussian vectors [V, N_channels, H, W] for views of one
    resolution (views as for pvg_render_views); feats: float32 [n,
    N_channels] on the parameters' device, each Gaussian's vector contiguous
    (the rows the compositing reads; the semantic class scores of Sec. 4.1;
    the cross-entropy against 2D labels is the caller's).
    Differentiable in feats and the parameters."""
    full = _full_views(views)
    if len({(int(v[0]["width"]), int(v[0]["height"])) for v in full}) != 1:
        raise ValueError("views of one resolution are required")
    return PVGRenderSemantic.apply(full, feats.contiguous(), *params)
