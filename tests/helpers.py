"""Helpers of the GPU parity tests: run the HIP path and the oracle on the
same seeded inputs and compare them."""
from __future__ import annotations

import numpy as np

FIELDS = ("mu", "scale", "rot", "sh", "opacity", "vel", "period", "tau", "beta")


def to_device(scene, device="cuda"):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(scene[f])).to(device) for f in FIELDS]


def gpu_forward(scene, cam, t, dt=0.0, mode=0, bg=(0.0, 0.0, 0.0), params=None, tile_cull=True):
    """The HIP forward; returns numpy copies of every stage's output.  "M" is
    the rectangle instance count, "L" the number of listed (sorted) ones."""
    import torch
    import paper_2311_18561_amd as pvg
    params = to_device(scene) if params is None else params
    img, T, nc, geom, bins = pvg.render(params, cam, t, dt, mode, bg, tile_cull=tile_cull)
    torch.cuda.synchronize()
    M = bins.num_instances
    L = bins.num_listed()
    return {
        "img": img.cpu().numpy(), "final_T": T.cpu().numpy(), "n_contrib": nc.cpu().numpy(),
        "xy": geom.xy.cpu().numpy(), "depth": geom.depth.cpu().numpy(), "conic_op": geom.conic_op.cpu().numpy(),
        "rgb": geom.rgb.cpu().numpy(), "radius": geom.radius.cpu().numpy(),
        "tiles": geom.tiles.cpu().numpy().view(np.uint32),
        "M": M, "L": L, "num_visible": bins.num_visible,
        "keys": bins.keys[:L].cpu().numpy().view(np.uint32), "vals": bins.vals[:L].cpu().numpy().view(np.uint32),
        "ranges": bins.ranges.cpu().numpy().view(np.uint32),
        "_geom": geom, "_bins": bins, "_params": params,
    }


def last_contributor_ids(n_contrib, vals, ranges, width):
    """Index of each pixel's last contributing Gaussian (-1 if none): the list
    position n_contrib - 1 looked up in its tile's list.  It does not depend on
    which non-contributing entries a list holds."""
    H, W = n_contrib.shape
    GX = (width + 15) // 16
    ys, xs = np.mgrid[0:H, 0:W]
    tile = (ys // 16) * GX + (xs // 16)
    rng = np.asarray(ranges, np.int64).reshape(-1, 2)
    pos = rng[tile, 0] + n_contrib.astype(np.int64) - 1
    out = np.full((H, W), -1, np.int64)
    has = n_contrib > 0
    out[has] = np.asarray(vals, np.int64)[pos[has]]
    return out


def check_culled_lists(culled_keys, culled_vals, culled_ranges, rect_tile, rect_gauss, pre, cam, n, sample=None):
    """A culled list is valid when (1) it is the rectangle list with entries
    removed, order kept, (2) its ranges delimit its tiles, and (3) every
    removed (tile, Gaussian) entry is one that each pixel of the tile skips
    (power > 0 or alpha < 1/255, evaluated in FP64; on a seeded sample of
    `sample` removed entries if given).  Returns the count removed."""
    W, H = cam["width"], cam["height"]
    GX = (W + 15) // 16
    ck = np.asarray(culled_keys, np.int64) * (n + 1) + np.asarray(culled_vals, np.int64)
    rk = np.asarray(rect_tile, np.int64) * (n + 1) + np.asarray(rect_gauss, np.int64)
    order = np.argsort(rk, kind="stable")
    pos = np.searchsorted(rk[order], ck)
    assert np.all(pos < rk.size) and np.array_equal(rk[order][np.minimum(pos, rk.size - 1)], ck), "entry not listed"
    ridx = order[pos]
    assert np.all(np.diff(ridx) > 0), "order of the rectangle list not kept"
    rng = np.asarray(culled_ranges, np.int64).reshape(-1, 2)
    tiles = np.asarray(culled_keys, np.int64)
    for t in np.unique(tiles):
        a, b = np.searchsorted(tiles, t), np.searchsorted(tiles, t, side="right")
        assert rng[t, 0] == a and rng[t, 1] == b
    keep = np.zeros(rk.size, bool)
    keep[ridx] = True
    drop = np.nonzero(~keep)[0]
    n_drop = int(drop.size)
    if sample is not None and drop.size > sample:
        drop = np.sort(np.random.default_rng(11).choice(drop, sample, replace=False))
    xy = pre["xy"].astype(np.float64)
    co = pre["conic_op"].astype(np.float64)
    py, px = np.mgrid[0:16, 0:16]
    for s in range(0, drop.size, 4096):
        d = drop[s:s + 4096]
        t = np.asarray(rect_tile, np.int64)[d]
        g = np.asarray(rect_gauss, np.int64)[d]
        X = (t % GX)[:, None] * 16 + px.reshape(1, -1)
        Y = (t // GX)[:, None] * 16 + py.reshape(1, -1)
        inside = (X < W) & (Y < H)
        dx = xy[g, 0][:, None] - X
        dy = xy[g, 1][:, None] - Y
        A, B, C, op = co[g, 0][:, None], co[g, 1][:, None], co[g, 2][:, None], co[g, 3][:, None]
        power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
        alpha = np.minimum(0.99, op * np.exp(np.minimum(power, 0.0)))
        skipped = (power > 0) | (alpha < 1.0 / 255.0) | ~inside
        assert np.all(skipped), "a removed entry would contribute"
    return n_drop


def geom_as_oracle_pre(g, cam):
    """The GPU's per-Gaussian record in the oracle's layout (rect recomputed
    by the oracle's own rule from xy and radius is not needed: the oracle's
    bin sort takes rect, which we derive the same way the definition does)."""
    import math
    n = g["radius"].shape[0]
    GX, GY = (cam["width"] + 15) // 16, (cam["height"] + 15) // 16
    rect = np.zeros((n, 4), np.int32)
    x = g["xy"][:, 0].astype(np.float32)
    y = g["xy"][:, 1].astype(np.float32)
    r = g["radius"].astype(np.float32)
    sixteen, fifteen = np.float32(16.0), np.float32(15.0)
    with np.errstate(invalid="ignore"):
        rect[:, 0] = np.clip(np.floor((x - r) / sixteen), 0, GX)
        rect[:, 1] = np.clip(np.floor((y - r) / sixteen), 0, GY)
        rect[:, 2] = np.clip(np.floor(((x + r) + fifteen) / sixteen), 0, GX)
        rect[:, 3] = np.clip(np.floor(((y + r) + fifteen) / sixteen), 0, GY)
    rect[g["radius"] <= 0] = 0
    del math
    return {"xy": g["xy"], "depth": g["depth"], "conic_op": g["conic_op"], "rgb": g["rgb"],
            "radius": g["radius"], "rect": rect, "tiles": g["tiles"], "flags": np.zeros(n, np.uint32)}


def grad_tolerance_report(g_gpu, g_ref, rel=1e-3, floor=1e-2, magnitude=None):
    """Per element |g - g*| <= rel * max(|g*|, floor * rms(g*)); returns (worst ratio, l2 rel err).
    magnitude (optional, same shape): the scale of the terms summed into g*
    (for a sum over views, the sum of the views' |g*|), used instead of |g*|,
    since FP32 sums are accurate relative to their terms, not to the total."""
    g_gpu = np.asarray(g_gpu, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    rms = np.sqrt(np.mean(g_ref ** 2)) if g_ref.size else 0.0
    mag = np.abs(g_ref) if magnitude is None else np.maximum(np.abs(g_ref), np.asarray(magnitude, np.float64))
    denom = np.maximum(mag, floor * rms)
    denom = np.where(denom > 0, denom, 1.0)
    ratio = np.abs(g_gpu - g_ref) / (rel * denom)
    l2 = np.linalg.norm(g_gpu - g_ref) / max(np.linalg.norm(g_ref), 1e-300)
    return float(ratio.max() if ratio.size else 0.0), float(l2)
