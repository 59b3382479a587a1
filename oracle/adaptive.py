"""Oracle of the position-aware adaptive control (Sec. 3.3, Eq. (9), and the
split rules in the implementation details of the appendix).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, one
step of the rule set after another.  The clone / split / prune decisions
are taken in FP32, the precision of the kernels they check; each FP32
expression is evaluated one rounded operation at a time, in the order
written.  Parity is pinned by the tests in ``tests/test_oracle_densify.py``.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def gamma(mu, r):
    """Eq. (9): 1 inside twice the scene radius, |mu| / r - 1 outside; mu [3, N]."""
    x, y, z = (np.asarray(mu[k], f32) for k in range(3))
    nrm = np.sqrt((x * x + y * y) + z * z)
    r = f32(r)
    return np.where(nrm < f32(2.0) * r, f32(1.0), nrm / r - f32(1.0)).astype(f32)


def _quat_matrix(rot):
    """Rotation of the normalised quaternion (w, x, y, z), entries [3][3][N]."""
    qw, qx, qy, qz = (np.asarray(rot[k], f32) for k in range(4))
    qn = np.sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz)
    w, x, y, z = qw / qn, qx / qn, qy / qn, qz / qn
    one, two = f32(1.0), f32(2.0)
    return [[one - two * (y * y + z * z), two * (x * y - w * z), two * (x * z + w * y)],
            [two * (x * y + w * z), one - two * (x * x + z * z), two * (y * z - w * x)],
            [two * (x * z - w * y), two * (y * z + w * x), one - two * (x * x + y * y)]]


def split_child(sc, noise, k, cfg):
    """Child k (0 or 1) of every Gaussian: scale decay * s; dtau = beta eps_k3;
    tau + dtau; beta * beta_decay; mean mu + R(q) (s * eps_k) + dtau v~ with
    v~ = v exp(-beta / (2 l)) (Eq. (10)); exp in FP64, rounded once."""
    R = _quat_matrix(sc["rot"])
    s = np.asarray(sc["scale"], f32)
    eps = np.asarray(noise, f32)
    a = [s[d] * eps[4 * k + d] for d in range(3)]
    beta, l = np.asarray(sc["beta"], f32), np.asarray(sc["period"], f32)
    e = np.exp((-(beta / (f32(2.0) * l))).astype(np.float64)).astype(f32)
    dtau = beta * eps[4 * k + 3]
    mu = np.empty_like(np.asarray(sc["mu"], f32))
    for d in range(3):
        off = (R[d][0] * a[0] + R[d][1] * a[1]) + R[d][2] * a[2]
        vb = np.asarray(sc["vel"][d], f32) * e
        mu[d] = (np.asarray(sc["mu"][d], f32) + off) + dtau * vb
    return {"mu": mu, "scale": f32(cfg["split_scale_decay"]) * s,
            "tau": np.asarray(sc["tau"], f32) + dtau, "beta": f32(cfg["split_beta_decay"]) * beta}


def _pruned(mu, scale, opacity, cfg):
    smax = np.maximum(np.maximum(scale[0], scale[1]), scale[2])
    return (smax > f32(cfg["prune_scale"]) * gamma(mu, cfg["scene_radius"])) | (opacity < f32(cfg["min_opacity"]))


def plan(sc, accum, count, noise, cfg):
    """Per Gaussian the outputs that survive: (keep original, keep clone,
    keep child 0, keep child 1), each a bool [N]."""
    mu, s = np.asarray(sc["mu"], f32), np.asarray(sc["scale"], f32)
    o = np.asarray(sc["opacity"], f32)
    accum, count = np.asarray(accum, f32), np.asarray(count, f32)
    safe = np.where(count > 0, count, f32(1.0))
    avg = np.where(count > 0, accum / safe, f32(0.0))
    dens = avg >= f32(cfg["grad_threshold"])
    smax = np.maximum(np.maximum(s[0], s[1]), s[2])
    clone = dens & (smax <= f32(cfg["clone_scale"]) * gamma(mu, cfg["scene_radius"]))
    split = dens & ~clone
    keep = ~_pruned(mu, s, o, cfg)
    kids = []
    for k in range(2):
        ch = split_child(sc, noise, k, cfg)
        kids.append(split & ~_pruned(ch["mu"], ch["scale"], o, cfg))
    return (~split) & keep, clone & keep, kids[0], kids[1]


ROWS = {"mu": 3, "scale": 3, "rot": 4, "opacity": 1, "vel": 3, "period": 1, "tau": 1, "beta": 1}


def densify(sc, accum, count, noise, cfg, extra=None):
    """The pass: returns (new scene dict, new extra rows or None).  Order:
    parents by index; within a parent the original, its clone, child 0,
    child 1.  Extra rows [R, N] are kept for a surviving original and zero
    for every new Gaussian."""
    keep0, keep1, keep2, keep3 = plan(sc, accum, count, noise, cfg)
    kids = [split_child(sc, noise, k, cfg) for k in range(2)]
    n = int(sc["n"])
    src = []  # output column -> (parent, slot)
    for i in range(n):
        for slot, kp in enumerate((keep0, keep1, keep2, keep3)):
            if kp[i]:
                src.append((i, slot))
    m = len(src)
    par = np.array([p for p, _ in src], np.int64)
    slot = np.array([q for _, q in src], np.int64)
    out = {"n": m, "sh_degree": sc["sh_degree"]}
    for f in ("rot", "vel", "opacity", "period"):
        a = np.asarray(sc[f], f32)
        out[f] = a[..., par].copy()
    out["sh"] = np.asarray(sc["sh"], f32)[..., par].copy()
    for f in ("mu", "scale", "tau", "beta"):
        a = np.asarray(sc[f], f32)[..., par].copy()
        for k in range(2):
            sel = slot == 2 + k
            a[..., sel] = kids[k][f][..., par[sel]]
        out[f] = a
    ex = None
    if extra is not None:
        extra = np.asarray(extra, f32)
        ex = np.where((slot == 0)[None, :], extra[:, par], f32(0.0)).astype(f32)
    return out, ex


def view_space_stats(g2d_views, visible_views, sizes):
    """The statistics the adjoint accumulates: for each view in which a
    Gaussian is visible, |(W/2 dL/dx, H/2 dL/dy)| (its 2D mean's gradient in
    normalized device coordinates) and a count of 1.  g2d_views: per view
    [N, >= 2] screen-space gradients in pixels; visible_views: per view bool
    [N]; sizes: per view (W, H).  FP64."""
    n = len(visible_views[0])
    acc, cnt = np.zeros(n), np.zeros(n)
    for g, vis, (W, H) in zip(g2d_views, visible_views, sizes):
        gx = np.asarray(g[:, 0], np.float64) * (W / 2.0)
        gy = np.asarray(g[:, 1], np.float64) * (H / 2.0)
        acc += np.where(vis, np.hypot(gx, gy), 0.0)
        cnt += vis
    return acc, cnt


def split_by_staticness(sc, threshold):
    """Static / dynamic partition (Sec. 3.2): rho = beta / l in FP32, static
    when rho >= threshold; both parts in index order."""
    rho = np.asarray(sc["beta"], f32) / np.asarray(sc["period"], f32)
    st = rho >= f32(threshold)
    parts = []
    for mask in (st, ~st):
        idx = np.nonzero(mask)[0]
        part = {"n": int(idx.size), "sh_degree": sc["sh_degree"]}
        for f in ("mu", "scale", "rot", "sh", "opacity", "vel", "period", "tau", "beta"):
            part[f] = np.asarray(sc[f], f32)[..., idx].copy()
        parts.append(part)
    return parts[0], parts[1]
