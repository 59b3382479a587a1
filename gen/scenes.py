"""Synthetic scenes, cameras and request traces shaped like the paper's driving
workloads (Waymo front cameras, about 1M initial points, a ~30 m foreground
radius with a far field behind it; Sec. 4 implementation details).

No dataset item is used or reproduced; these draws stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

FIELDS = ("mu", "scale", "rot", "sh", "opacity", "vel", "period", "tau", "beta")

# focal length as a fraction of the image width (fx = 100 at W = 128)
FOCAL_PER_WIDTH = 100.0 / 128.0


@dataclass(frozen=True)
class SceneSpec:
    n: int
    sh_degree: int
    layout: str          # "box": means in a box in front of the camera; "path": around a 100 m path
    far_fraction: float  # fraction of "path" points drawn as a far field (config 4)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _draw_means(rng, spec: SceneSpec, log_scale_far):
    n = spec.n
    if spec.layout == "box":
        xy = rng.uniform(-5.0, 5.0, size=(2, n))
        z = rng.uniform(2.0, 12.0, size=(1, n))
        return np.concatenate([xy, z], axis=0), None
    # "path": a uniform point on the segment (0,0,0)-(0,0,100) plus a random
    # direction times a log-uniform distance.
    u = rng.uniform(0.0, 1.0, size=n)
    d = rng.standard_normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    sel = rng.uniform(0.0, 1.0, size=n)
    lo = np.where(sel < 0.7, math.log(1.0), math.log(30.0))
    hi = np.where(sel < 0.7, math.log(30.0), math.log(300.0))
    far = None
    if spec.far_fraction > 0.0:
        far = rng.uniform(0.0, 1.0, size=n) < spec.far_fraction
        lo = np.where(far, math.log(100.0), lo)
        hi = np.where(far, math.log(1000.0), hi)
    dist = np.exp(rng.uniform(0.0, 1.0, size=n) * (hi - lo) + lo)
    mu = d * dist
    mu[2] += 100.0 * u
    return mu, far


def make_scene(n: int, seed: int, sh_degree: int = 0, layout: str = "box",
               far_fraction: float = 0.0) -> dict:
    """Draw one scene of ``n`` Gaussians (float32 SoA arrays, see module doc)."""
    spec = SceneSpec(int(n), int(sh_degree), layout, float(far_fraction))
    rng = np.random.default_rng(seed)
    mu, far = _draw_means(rng, spec, None)
    log_s = rng.normal(-2.0, 0.5, size=(3, spec.n))
    if far is not None:
        log_s_far = rng.normal(0.0, 0.5, size=(3, spec.n))
        log_s = np.where(far[None, :], log_s_far, log_s)
    q = rng.standard_normal(size=(4, spec.n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    o = 1.0 / (1.0 + np.exp(-rng.standard_normal(size=spec.n)))
    v = rng.normal(0.0, 0.1, size=(3, spec.n))
    period = rng.uniform(0.5, 3.0, size=spec.n)
    tau = rng.uniform(0.0, 1.0, size=spec.n)
    beta = np.exp(rng.uniform(math.log(0.05), 0.0, size=spec.n))
    k = (spec.sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.2, size=(k, 3, spec.n))
    return {
        "n": spec.n,
        "sh_degree": spec.sh_degree,
        "mu": _f32(mu),
        "scale": _f32(np.exp(log_s)),
        "rot": _f32(q),
        "sh": _f32(sh),
        "opacity": _f32(o),
        "vel": _f32(v),
        "period": _f32(period),
        "tau": _f32(tau),
        "beta": _f32(beta),
    }


def subset_scene(scene: dict, idx) -> dict:
    """The Gaussians ``idx`` of ``scene`` as a scene of their own."""
    idx = np.asarray(idx)
    out = {"n": int(idx.size), "sh_degree": scene["sh_degree"]}
    for f in FIELDS:
        out[f] = np.ascontiguousarray(scene[f][..., idx])
    return out


def make_camera(width: int, height: int, R=None, center=(0.0, 0.0, 0.0),
                fx: float | None = None, znear: float = 0.2) -> dict:
    """Pinhole camera: x_cam = R x_world + T, looking down +z, x right, y down."""
    R = np.eye(3) if R is None else np.asarray(R, dtype=np.float64)
    c = np.asarray(center, dtype=np.float64)
    T = -R @ c
    f = FOCAL_PER_WIDTH * width if fx is None else float(fx)
    return {
        "R": R.astype(np.float32),
        "T": T.astype(np.float32),
        "fx": float(np.float32(f)),
        "fy": float(np.float32(f)),
        "cx": width / 2.0,
        "cy": height / 2.0,
        "width": int(width),
        "height": int(height),
        "znear": float(np.float32(znear)),
    }


def yaw_camera(width: int, height: int, yaw_deg: float, center) -> dict:
    """Camera at ``center`` turned by ``yaw_deg`` about the world y axis."""
    a = math.radians(yaw_deg)
    r_wc = np.array([[math.cos(a), 0.0, math.sin(a)],
                     [0.0, 1.0, 0.0],
                     [-math.sin(a), 0.0, math.cos(a)]])
    return make_camera(width, height, R=r_wc.T, center=center)


def make_target(width: int, height: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed + 1000)
    return _f32(rng.uniform(0.0, 1.0, size=(3, height, width)))


CONFIGS = {
    # forward only: 2,000 Gaussians, 128x96, SH degree 0
    0: dict(n=2000, seed=0, sh_degree=0, layout="box", width=128, height=96, views=1),
    # forward+backward: 200k Gaussians, 960x640, SH degree 3, L1 vs uniform target
    1: dict(n=200_000, seed=1, sh_degree=3, layout="box", width=960, height=640, views=1),
    # training-shaped step: 1M Gaussians, 1920x1280, 3 yawed cameras + second render at t+dt
    2: dict(n=1_000_000, seed=2, sh_degree=3, layout="path", width=1920, height=1280,
            views=3, dt=0.05),
    # large: 6M Gaussians, 40% far field, 6 cameras
    4: dict(n=6_000_000, seed=4, sh_degree=3, layout="path", width=1920, height=1280,
            views=6, far_fraction=0.4),
}


def make_config(cfg: int, n: int | None = None) -> dict:
    """Scene, cameras, render time and targets of one numbered workload.

    ``n`` overrides the Gaussian count (same distributions, same seed)."""
    c = dict(CONFIGS[cfg])
    if n is not None:
        c["n"] = int(n)
    scene = make_scene(c["n"], c["seed"], c["sh_degree"], c["layout"], c.get("far_fraction", 0.0))
    rng = np.random.default_rng(c["seed"] + 500)
    w, h = c["width"], c["height"]
    if c["layout"] == "box":
        t = 0.5
        cams = [make_camera(w, h)]
    else:
        t = float(np.float32(rng.uniform(0.0, 1.0)))
        center = (0.0, 0.0, 100.0 * t)
        yaws = [-45.0, 0.0, 45.0] if c["views"] == 3 else [0.0, 60.0, -60.0, 120.0, -120.0, 180.0]
        cams = [yaw_camera(w, h, y, center) for y in yaws]
    targets = [make_target(w, h, c["seed"] + i) for i in range(len(cams))]
    return {"cfg": cfg, "scene": scene, "cameras": cams, "t": t, "dt": c.get("dt", 0.0),
            "targets": targets, "width": w, "height": h}


RES_CLASSES = ((640, 480), (960, 640), (1920, 1280))


def make_trace(seed: int = 3, rate: float = 200.0, duration: float = 20.0, n_scenes: int = 4):
    """Poisson request stream on a 100 m straight path.

    Each request: arrival time (s), scene index, camera (yaw ~ U[-45,45] deg,
    centre uniform on the path), render time t ~ U[0,1], resolution class."""
    rng = np.random.default_rng(seed)
    reqs = []
    clock = 0.0
    while True:
        clock += rng.exponential(1.0 / rate)
        if clock >= duration:
            break
        scene = int(rng.integers(0, n_scenes))
        u = float(rng.uniform(0.0, 1.0))
        yaw = float(rng.uniform(-45.0, 45.0))
        t = float(np.float32(rng.uniform(0.0, 1.0)))
        res = int(rng.integers(0, len(RES_CLASSES)))
        w, h = RES_CLASSES[res]
        reqs.append({"arrival": clock, "scene": scene, "t": t, "res": res,
                     "camera": yaw_camera(w, h, yaw, (0.0, 0.0, 100.0 * u))})
    return reqs
