"""Python face of the continuous-batching render server (include/pvg_serve.h).

    srv = Server(max_batch=8, max_inflight=2)
    sid = srv.load_scene(params)            # nine float32 device tensors (SoA layout)
    img = torch.empty(3, H, W, device="cuda")
    tk = srv.submit(sid, cam, t, img)       # returns at once
    res = srv.wait(tk)                      # img now holds the render

All scheduling and rendering run in libpvg; this module marshals arguments.
"""
from __future__ import annotations

import ctypes as C

from . import _lib as L
from .render import _check_params, camera_struct, gaussians_struct


class Server:
    def __init__(self, max_batch=8, max_inflight=2, use_graphs=True, mem_budget_bytes=0,
                 max_batch_gaussians=16_000_000, max_batch_pixels=16 * 1920 * 1280, instance_capacity=1 << 29,
                 device=0, stub_launch_us=0):
        cfg = L.ServeConfig()
        cfg.device, cfg.max_batch, cfg.max_inflight = int(device), int(max_batch), int(max_inflight)
        cfg.use_graphs = 1 if use_graphs else 0
        cfg.mem_budget_bytes = int(mem_budget_bytes)
        cfg.max_batch_gaussians = int(max_batch_gaussians)
        cfg.max_batch_pixels = int(max_batch_pixels)
        cfg.instance_capacity = int(instance_capacity)
        cfg.stub_launch_us = int(stub_launch_us)
        self._lib = L.load()
        h = C.c_void_p()
        L.check(self._lib.pvg_serve_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._keep = {}  # tickets -> destination tensors (kept alive until waited)

    def load_scene(self, params=None, n=None, sh_degree=0) -> int:
        """Copies a scene into server memory.  With the stub launcher, n and
        sh_degree describe a scene that is never read."""
        if params is not None:
            params, n, degree = _check_params(params)
            g = gaussians_struct(params, n, degree)
        else:
            g = L.Gaussians()
            g.n, g.sh_degree = int(n), int(sh_degree)
            dummy = C.c_void_p(1)
            for f in ("mu", "scale", "rot", "sh", "opacity", "vel", "period", "tau", "beta"):
                setattr(g, f, dummy.value)
        sid = C.c_int32()
        L.check(self._lib.pvg_serve_load_scene(self._h, C.byref(g), C.byref(sid)))
        return sid.value

    def unload_scene(self, sid: int):
        L.check(self._lib.pvg_serve_unload_scene(self._h, int(sid)))

    def submit(self, scene_id, cam: dict, t, dst=None, bg=(0.0, 0.0, 0.0), tag=0) -> int:
        r = L.Request()
        r.scene_id = int(scene_id)
        r.camera = camera_struct(cam)
        r.t = float(t)
        r.bg[:] = [float(b) for b in bg]
        r.dst = dst.data_ptr() if dst is not None else None
        r.user_tag = int(tag)
        tk = C.c_uint64()
        L.check(self._lib.pvg_serve_submit(self._h, C.byref(r), C.byref(tk)))
        if dst is not None:
            self._keep[tk.value] = dst
        return tk.value

    def wait(self, ticket: int, timeout_s: float | None = None) -> L.Result:
        res = L.Result()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        L.check(self._lib.pvg_serve_wait(self._h, C.c_uint64(ticket), us, C.byref(res)))
        return res

    def poll(self, ticket: int) -> bool:
        d = C.c_int32()
        L.check(self._lib.pvg_serve_poll(self._h, C.c_uint64(ticket), C.byref(d)))
        return bool(d.value)

    def release(self, ticket: int):
        L.check(self._lib.pvg_serve_release(self._h, C.c_uint64(ticket)))
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        r = L.ServeReport()
        L.check(self._lib.pvg_serve_stats(self._h, C.byref(r)))
        return {f: getattr(r, f) for f, _ in L.ServeReport._fields_}

    def reset_stats(self):
        L.check(self._lib.pvg_serve_reset_stats(self._h))

    def close(self):
        if self._h is not None:
            L.check(self._lib.pvg_serve_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
