"""Helpers of the GPU parity tests: run the HIP path and the oracle on the
same seeded inputs and compare them."""
from __future__ import annotations

import os
import tempfile

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


def grad_tolerance_report(g_gpu, g_ref, rel=1e-3, floor=1e-2, magnitude=None, terms=None):
    """Per element |g - g*| <= rel * max(|g*|, floor * rms(g*)); returns (worst ratio, l2 rel err).
    magnitude (optional, same shape): the scale of the terms summed into g*
    (for a sum over views, the sum of the views' |g*|), used instead of |g*|,
    since FP32 sums are accurate relative to their terms, not to the total.
    terms (optional, same shape): the oracle's bound on the magnitude of the
    per-pixel terms behind each element (oracle.grad_magnitude_f64); the bar
    is then at least rel * 1e-2 * terms, about 170 FP32 roundings of that
    scale, which a sum of a few hundred rounded terms can reach but a wrong
    term cannot hide under where the element does not cancel."""
    g_gpu = np.asarray(g_gpu, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    rms = np.sqrt(np.mean(g_ref ** 2)) if g_ref.size else 0.0
    mag = np.abs(g_ref) if magnitude is None else np.maximum(np.abs(g_ref), np.asarray(magnitude, np.float64))
    if terms is not None:
        mag = np.maximum(mag, 1e-2 * np.asarray(terms, np.float64))
    denom = np.maximum(mag, floor * rms)
    denom = np.where(denom > 0, denom, 1.0)
    ratio = np.abs(g_gpu - g_ref) / (rel * denom)
    l2 = np.linalg.norm(g_gpu - g_ref) / max(np.linalg.norm(g_ref), 1e-300)
    return float(ratio.max() if ratio.size else 0.0), float(l2)


_EXP_VARIANTS = {}


def oracle_exp_variants():
    """Two builds of the oracle whose per-pair exponential in the FP32 image
    is one ulp above and one ulp below the C library's expf.  Each side's FP32
    exp may differ from the other's by an ulp (the GPU uses its own device
    exponential), and where a pair's alpha sits within that of 1/255 the two
    admissible roundings skip or blend it, moving the pixel by up to about
    T c / 255.  The image oracles of the three builds bound the set of
    correct FP32 results for such pixels."""
    import oracle
    if not _EXP_VARIANTS:
        src = oracle.source_text()
        old = "    const float alpha = std::min(0.99f, d.op * std::exp(power));"
        assert src.count(old) == 1, "the oracle's FP32 blend line changed"
        for name, towards in (("up", "2.0f"), ("down", "0.0f")):
            new = f"    const float alpha = std::min(0.99f, d.op * std::nextafter(std::exp(power), {towards}));"
            path = os.path.join(tempfile.gettempdir(), f"liboracle_exp_{name}_{os.getpid()}.so")
            _EXP_VARIANTS[name] = oracle.build_variant(src.replace(old, new), path)
    return dict(_EXP_VARIANTS)


def oracle_image_set(scene, cam, t, dt=0.0, mode=0, bg=(0.0, 0.0, 0.0)):
    """The FP32 oracle image with the C library's expf and with the two
    one-ulp variants (see oracle_exp_variants): [3, 3, H, W]."""
    import oracle
    imgs = [oracle.render(scene, cam, t, dt, mode, bg)["img"]]
    for path in oracle_exp_variants().values():
        with oracle.use_library(path):
            imgs.append(oracle.render(scene, cam, t, dt, mode, bg)["img"])
    return np.stack(imgs)


def image_in_set_error(img, refs):
    """(max over pixels of the smallest per-pixel error against any image of
    the set, pixels whose error against refs[0] alone exceeds 1e-4)."""
    per = np.abs(np.asarray(img)[None] - refs).max(axis=1)  # [variants, H, W]
    return float(per.min(axis=0).max()), int((per[0] > 1e-4).sum())


def oracle_margin(pre, bins, cam, t, dt=0.0, mode=0, bg=(0.0, 0.0, 0.0), tiles=None, gradients=False):
    """The oracle's per-pixel decision margin (oracle.render_margin_f32):
    below 1 a skip or stop decision of the pixel's walk (with gradients also
    the adjoint's alpha-clamp branch) sits within the rounding a
    differently-rounded FP32 renderer may resolve the other way."""
    import oracle
    return oracle.render_margin_f32(pre, bins, cam, t, dt, mode, bg, tiles, gradients)


def oracle_margin_tiles(pre, bins, cam, t, dt, tile_ids, gradients=False, mode=0, bg=(0.0, 0.0, 0.0)):
    """oracle_margin over the listed tiles only (+inf elsewhere)."""
    out = None
    for tid in tile_ids:
        m = oracle_margin(pre, bins, cam, t, dt, mode, bg, (int(tid), int(tid) + 1), gradients)
        out = m if out is None else np.minimum(out, m)
    return out


def unambiguous(margin):
    """0/1 weights that drop the pixels with an ambiguous decision from a
    loss, so that neither side's gradient depends on how it resolved them."""
    return (np.asarray(margin) >= 1.0).astype(np.float32)


def image_parity(img, ref, margin, tol=1e-4, rows=None, max_excused=None):
    """Compares an FP32 image (or any [C,H,W] / [H,W] per-pixel result) with
    the oracle's: every pixel whose decisions are unambiguous (margin >= 1)
    within `tol`; a pixel whose skip or stop decision is ambiguous may take
    either branch, so it is excused from the bar (both results are correct
    FP32 renders of the definition); their number is bounded by
    `max_excused` (default: 1e-4 of the pixels, at least 2).  rows: an
    optional row slice to compare.  Returns (worst error at unambiguous
    pixels, pixels excused)."""
    img = np.asarray(img, np.float64)
    ref = np.asarray(ref, np.float64)
    if img.ndim == 2:
        img, ref = img[None], ref[None]
    m = np.asarray(margin)
    if rows is not None:
        img, ref, m = img[:, rows], ref[:, rows], m[rows]
    err = np.abs(img - ref).max(axis=0)
    amb = m < 1.0
    worst = float(err[~amb].max()) if (~amb).any() else 0.0
    excused = int(((err > tol) & amb).sum())
    bound = max(2, int(1e-4 * m.size)) if max_excused is None else max_excused
    assert worst <= tol, f"error {worst:.3g} above {tol} at a pixel whose decisions are unambiguous"
    assert excused <= bound, f"{excused} pixels differ at ambiguous decisions (bound {bound})"
    return worst, excused


def oracle_grads(orc, sc64, cam, t, dt, mode, bg, pre, bins, dimg, **kw):
    """The FP64 adjoint (backward_f64) and, per parameter entry, the
    magnitude of its terms: (grads, g2d, terms)."""
    return orc.backward_f64(sc64, cam, t, dt, mode, bg, pre, bins, dimg, want_terms=True, **kw)
