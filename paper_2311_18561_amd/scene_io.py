"""Scene files: one raw float32 ``.npy`` per parameter field, in the SoA layout
the library reads (mu [3, n], scale [3, n], rot [4, n], sh [K, 3, n],
opacity [n], vel [3, n], period [n], tau [n], beta [n]; K = (degree + 1)^2).

    save_scene("scene_dir", params)          # params: nine tensors or arrays
    params = load_scene("scene_dir", "cuda") # nine contiguous float32 tensors
    sid = server.load_scene(params)          # into a render server's memory

Files are written and read with numpy's own format (no pickling); a scene
is checked for matching n, shapes and dtype before it is returned.
"""
from __future__ import annotations

import os

import numpy as np

FIELDS = ("mu", "scale", "rot", "sh", "opacity", "vel", "period", "tau", "beta")
_ROWS = {"mu": 3, "scale": 3, "rot": 4, "vel": 3}


def _check(arrays: dict) -> int:
    n = arrays["mu"].shape[-1]
    for f in FIELDS:
        a = arrays[f]
        if a.dtype != np.float32:
            raise ValueError(f"{f} must be float32, got {a.dtype}")
        if f == "sh":
            ok = a.ndim == 3 and a.shape[0] in (1, 4, 9, 16) and a.shape[1:] == (3, n)
        elif f in _ROWS:
            ok = a.shape == (_ROWS[f], n)
        else:
            ok = a.shape == (n,)
        if not ok:
            raise ValueError(f"{f} has shape {a.shape}, which does not fit n = {n}")
    return n


def save_scene(path: str, params) -> None:
    """Writes <path>/<field>.npy for the nine fields (tensors on any device,
    or numpy arrays, in the order mu, scale, rot, sh, opacity, vel, period,
    tau, beta)."""
    arrays = {}
    for f, p in zip(FIELDS, params):
        a = p.detach().cpu().numpy() if hasattr(p, "detach") else np.asarray(p)
        arrays[f] = np.ascontiguousarray(a)
    if len(arrays) != len(FIELDS):
        raise ValueError(f"expected {len(FIELDS)} fields, got {len(arrays)}")
    _check(arrays)
    os.makedirs(path, exist_ok=True)
    for f, a in arrays.items():
        tmp = os.path.join(path, f + ".tmp.npy")
        np.save(tmp, a, allow_pickle=False)
        os.replace(tmp, os.path.join(path, f + ".npy"))


def load_scene(path: str, device=None):
    """The nine fields of a saved scene: numpy arrays (device None) or
    contiguous float32 torch tensors on `device`."""
    arrays = {f: np.load(os.path.join(path, f + ".npy"), allow_pickle=False) for f in FIELDS}
    _check(arrays)
    if device is None:
        return [arrays[f] for f in FIELDS]
    import torch
    return [torch.from_numpy(arrays[f]).to(device).contiguous() for f in FIELDS]
