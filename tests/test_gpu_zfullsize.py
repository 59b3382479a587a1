"""The 1M-Gaussian, 1920x1280, degree-3 training-shaped workload at full size,
through the same call and launch configuration bench.py times: six views (3
cameras x {H(t), H^(t + 0.05)}) rendered by pvg_render_views (views on side
streams, lists kept for the backward, one multi-view per-Gaussian adjoint).

Forward: one full tile row of two views against the FP32 oracle (image,
transmittance, last contributor).  Backward: an image gradient confined to a
few random tiles of those two views, so the FP64 oracle adjoint restricted
to the same tiles gives the exact expected gradient of every parameter.
Pixels whose skip or stop decisions are ambiguous (the oracle's decision
margin below 1: either branch is a correct FP32 render) are held to no image
bar and get no loss weight.
"""
import numpy as np
import pytest

import gen
from helpers import (FIELDS, check_culled_lists, gpu_forward, grad_tolerance_report, image_parity,
                     last_contributor_ids, oracle_grads, oracle_margin, oracle_margin_tiles, to_device, unambiguous)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_training_workload_full_size_sampled(orc):
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(2)
    scene, cams, t, dt = cfg["scene"], cfg["cameras"], cfg["t"], cfg["dt"]
    W, H = cfg["width"], cfg["height"]
    GX, GY = (W + 15) // 16, (H + 15) // 16
    views = [(cam, t, d) for cam in cams for d in (0.0, dt)]
    checked = {2: (cams[1], 0.0), 3: (cams[1], dt)}  # the middle camera, both times
    rng = np.random.default_rng(12)
    masks, weights, oracle_lists = {}, {}, {}
    for k, (cam, d) in checked.items():
        pre = orc.preprocess_f32(scene, cam, t, d)
        bins = orc.bin_sort(pre, cam)
        oracle_lists[k] = (pre, bins)
        m = np.zeros(GX * GY, np.uint8)
        m[rng.choice(np.arange(GX * (GY // 4), GX * (3 * GY // 4)), 6, replace=False)] = 1
        keep = np.repeat(np.repeat(m.reshape(GY, GX), 16, 0), 16, 1)[:H, :W]
        keep = keep * unambiguous(oracle_margin_tiles(pre, bins, cam, t, d, np.nonzero(m)[0], gradients=True))
        masks[k] = m
        weights[k] = (rng.standard_normal((3, H, W)) * keep).astype(np.float32)
    params = [p.requires_grad_(True) for p in to_device(scene)]
    imgs = pvg.pvg_render_views(params, views)
    loss = sum((imgs[k] * torch.from_numpy(w).cuda()).sum() for k, w in weights.items())
    loss.backward()
    got = {f: p.grad.detach().cpu().numpy().astype(np.float64) for f, p in zip(FIELDS, params)}
    # the same images through the single-view path, for the contributor lists
    ref = {f: np.zeros_like(got[f]) for f in FIELDS}
    mag = {f: np.zeros_like(got[f]) for f in FIELDS}  # per view max(|g*|, 1e-2 of the terms), summed
    sc64 = orc.scene64(scene)
    row = GY // 2
    for k, (cam, d) in checked.items():
        pre, bins = oracle_lists[k]
        img_o, T_o, nc_o = orc.render_f32(pre, bins, cam, t, d, tiles=(row * GX, (row + 1) * GX))
        margin = oracle_margin(pre, bins, cam, t, d, tiles=(row * GX, (row + 1) * GX))
        ys = slice(row * 16, row * 16 + 16)
        g_img = imgs[k].detach().cpu().numpy()
        err, excused = image_parity(g_img, img_o, margin, rows=ys)
        print(f"[view {k}] tile row {row}: max |img - oracle| = {err:.3g} at unambiguous pixels, {excused} excused")
        # last contributor of each pixel of the row: the GPU's lists are culled, the oracle's are rectangles
        img_g, T_g, nc_g, geom_g, bins_g = pvg.render(params, cam, t, d)
        assert torch.equal(img_g, imgs[k].detach())
        L_ = bins_g.num_listed()
        ids_g = last_contributor_ids(nc_g.cpu().numpy(), bins_g.vals[:L_].cpu().numpy().view(np.uint32),
                                     bins_g.ranges.cpu().numpy().view(np.uint32), W)
        ids_o = last_contributor_ids(nc_o, bins["inst_gauss"], bins["ranges"], W)
        flips = ids_g[ys] != ids_o[ys]
        print(f"[view {k}] last-contributor differences in the row: {int(flips.sum())} of {16 * W}")
        assert not np.any(flips & (margin[ys] >= 1.0))
        image_parity(T_g.cpu().numpy(), T_o, margin, rows=ys)
        part, _, terms = oracle_grads(orc, sc64, cam, t, d, 0, (0, 0, 0), pre, bins, weights[k].astype(np.float64),
                                      tile_mask=masks[k])
        for f in FIELDS:
            ref[f] += part[f]
            mag[f] += np.maximum(np.abs(part[f]), 1e-2 * terms[f])
    touched = np.zeros(scene["n"], bool)
    for f in FIELDS:
        a = np.abs(ref[f]).reshape(-1, scene["n"]).max(axis=0)
        touched |= a > 0
    print(f"Gaussians with a nonzero reference gradient: {int(touched.sum())}")
    assert touched.sum() > 100
    # The tolerance floor (1e-2 rms of the tensor) is taken over the Gaussians
    # the masked tiles reach: over all 1M, mostly exact zeros, it would shrink
    # by the square root of the touched fraction (about 50x here).
    for f in FIELDS:
        n = scene["n"]
        g2 = got[f].reshape(-1, n)
        r2 = ref[f].reshape(-1, n)
        assert np.abs(g2[:, ~touched]).max() <= 1e-6 * np.abs(r2).max(), f
        worst, l2 = grad_tolerance_report(g2[:, touched], r2[:, touched], magnitude=mag[f].reshape(-1, n)[:, touched])
        j = np.unravel_index(np.argmax(np.abs(g2[:, touched] - r2[:, touched])), r2[:, touched].shape)
        print(f"[full size] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}; largest difference "
              f"{g2[:, touched][j]:.6g} vs {r2[:, touched][j]:.6g}")
        assert worst <= 1.0, f


def test_training_view_sort_full_size(orc):
    """The sorted lists of one whole 1920x1280 view of the 1M-Gaussian scene
    (the middle camera's H(t), about 31M rectangle instances), bit for bit:
    radii and tile counts, the rectangle lists (tile_cull=False: tile ids and
    Gaussian indices in (tile, depth, index) order) and the tile ranges
    against the oracle's sort; the culled lists as order-kept sublists whose
    dropped entries no pixel of their tile can use."""
    cfg = gen.make_config(2)
    scene, cam, t = cfg["scene"], cfg["cameras"][1], cfg["t"]
    pre = orc.preprocess_f32(scene, cam, t)
    bins = orc.bin_sort(pre, cam)
    gr = gpu_forward(scene, cam, t, tile_cull=False)
    print(f"[sort full size] rectangle instances: GPU {gr['M']}, oracle {bins['M']}; visible {gr['num_visible']}",
          flush=True)
    assert bins["M"] > 20_000_000
    assert np.array_equal(gr["radius"], pre["radius"])
    assert np.array_equal(gr["tiles"], pre["tiles"].view(np.uint32))
    assert gr["M"] == gr["L"] == bins["M"]
    assert np.array_equal(gr["keys"], bins["inst_tile"])
    assert np.array_equal(gr["vals"], bins["inst_gauss"])
    assert np.array_equal(gr["ranges"], bins["ranges"])
    del gr
    g = gpu_forward(scene, cam, t, tile_cull=True)
    dropped = check_culled_lists(g["keys"], g["vals"], g["ranges"], bins["inst_tile"], bins["inst_gauss"], pre, cam,
                                 scene["n"], sample=200_000)
    print(f"[sort full size] culled lists: {g['L']} listed, {dropped} rectangle entries dropped")
    assert g["L"] + dropped == bins["M"]


def test_large_scene_six_cameras_sampled(orc):
    """The 6M-Gaussian scene (40% far field) seen by six cameras, through the
    same multi-view call.  For two of the views, the oracle renders one tile
    row and differentiates a loss on a few tiles from the Gaussians whose
    rectangles reach those tiles (per-Gaussian preprocessing is independent
    and the subset keeps the index order, so those pixels' lists are exact)."""
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(4)
    scene, cams, t = cfg["scene"], cfg["cameras"], cfg["t"]
    W, H = cfg["width"], cfg["height"]
    GX, GY = (W + 15) // 16, (H + 15) // 16
    n = scene["n"]
    views = [(cam, t) for cam in cams]
    checked = (0, 3)
    rng = np.random.default_rng(21)
    row = GY // 2
    masks, weights, subsets = {}, {}, {}
    for k in checked:
        cam = cams[k]
        m = np.zeros(GX * GY, np.uint8)
        m[rng.choice(np.arange(GX * (GY // 4), GX * (3 * GY // 4)), 6, replace=False)] = 1
        pre = orc.preprocess_f32(scene, cam, t)
        r = pre["rect"]
        tile_ids = np.nonzero(m)[0]
        reach = (pre["radius"] > 0) & (r[:, 1] <= row) & (row < r[:, 3])
        for tid in tile_ids:
            tx, ty = tid % GX, tid // GX
            reach |= (pre["radius"] > 0) & (r[:, 0] <= tx) & (tx < r[:, 2]) & (r[:, 1] <= ty) & (ty < r[:, 3])
        idx = np.nonzero(reach)[0]
        sub = gen.subset_scene(scene, idx)
        pre_s = orc.preprocess_f32(sub, cam, t)
        assert np.array_equal(pre_s["radius"], pre["radius"][idx]) and np.array_equal(pre_s["xy"], pre["xy"][idx])
        bins_s = orc.bin_sort(pre_s, cam)
        subsets[k] = (idx, sub, pre_s, bins_s)
        keep = np.repeat(np.repeat(m.reshape(GY, GX), 16, 0), 16, 1)[:H, :W]
        keep = keep * unambiguous(oracle_margin_tiles(pre_s, bins_s, cam, t, 0.0, tile_ids, gradients=True))
        masks[k] = m
        weights[k] = (rng.standard_normal((3, H, W)) * keep).astype(np.float32)
    params = [p.requires_grad_(True) for p in to_device(scene)]
    imgs = pvg.pvg_render_views(params, views)
    loss = sum((imgs[k] * torch.from_numpy(w).cuda()).sum() for k, w in weights.items())
    loss.backward()
    got = {f: p.grad.detach().cpu().numpy().astype(np.float64).reshape(-1, n) for f, p in zip(FIELDS, params)}
    ref = {f: np.zeros_like(got[f]) for f in FIELDS}
    mag = {f: np.zeros_like(got[f]) for f in FIELDS}
    for k in checked:
        cam = cams[k]
        idx, sub, pre_s, bins_s = subsets[k]
        img_o, T_o, nc_o = orc.render_f32(pre_s, bins_s, cam, t, tiles=(row * GX, (row + 1) * GX))
        margin = oracle_margin(pre_s, bins_s, cam, t, tiles=(row * GX, (row + 1) * GX))
        ys = slice(row * 16, row * 16 + 16)
        err, excused = image_parity(imgs[k].detach().cpu().numpy(), img_o, margin, rows=ys)
        print(f"[6M view {k}] {idx.size} Gaussians reach the sampled tiles; tile row {row}: "
              f"max |img - oracle| = {err:.3g} at unambiguous pixels, {excused} excused")
        part, _, terms = oracle_grads(orc, orc.scene64(sub), cam, t, 0.0, 0, (0, 0, 0), pre_s, bins_s,
                                      weights[k].astype(np.float64), tile_mask=masks[k])
        for f in FIELDS:
            ref[f][:, idx] += part[f].reshape(-1, idx.size)
            mag[f][:, idx] += np.maximum(np.abs(part[f]), 1e-2 * terms[f]).reshape(-1, idx.size)
    touched = np.zeros(n, bool)
    for f in FIELDS:
        touched |= np.abs(ref[f]).max(axis=0) > 0
    print(f"Gaussians with a nonzero reference gradient: {int(touched.sum())}")
    assert touched.sum() > 100
    for f in FIELDS:
        assert np.abs(got[f][:, ~touched]).max() <= 1e-6 * np.abs(ref[f]).max(), f
        worst, l2 = grad_tolerance_report(got[f][:, touched], ref[f][:, touched], magnitude=mag[f][:, touched])
        print(f"[6M] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f


def test_channels_full_size_sampled(orc):
    """The channel step's render at the benchmark's shape: the six views of
    the 1M-Gaussian workload through pvg_render_views(channels=True,
    normalized_depth=True).  For the middle camera's flow-translated view:
    one tile row of the normalized depth, velocity and staticness maps
    against the oracle (pixels with unambiguous decisions), and a loss on
    normalized depth, opacity, velocity
    and staticness confined to six tiles against the FP64 adjoint on those
    tiles (the tolerance summed over the loss's sources: the quotient's two
    terms and the rest)."""
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(2)
    scene, cams, t, dt = cfg["scene"], cfg["cameras"], cfg["t"], cfg["dt"]
    W, H = cfg["width"], cfg["height"]
    GX, GY = (W + 15) // 16, (H + 15) // 16
    views = [(cam, t, d) for cam in cams for d in (0.0, dt)]
    k, cam, d = 3, cams[1], dt
    rng = np.random.default_rng(31)
    m = np.zeros(GX * GY, np.uint8)
    m[rng.choice(np.arange(GX * (GY // 4), GX * (3 * GY // 4)), 6, replace=False)] = 1
    pre = orc.preprocess_f32(scene, cam, t, d)
    bins = orc.bin_sort(pre, cam)
    keep = np.repeat(np.repeat(m.reshape(GY, GX), 16, 0), 16, 1)[:H, :W].astype(np.float64)
    keep = keep * unambiguous(oracle_margin_tiles(pre, bins, cam, t, d, np.nonzero(m)[0], gradients=True))
    wD = (0.05 * rng.standard_normal((H, W)) * keep).astype(np.float32)
    wO = (rng.standard_normal((H, W)) * keep).astype(np.float32)
    wF = (rng.standard_normal((4, H, W)) * keep).astype(np.float32)
    params = [p.requires_grad_(True) for p in to_device(scene)]
    img, dn, opac, vbar, rho = pvg.pvg_render_views(params, views, channels=True, normalized_depth=True)
    cu = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    loss = ((dn[k] * cu(wD)).sum() + (opac[k] * cu(wO)).sum() + (vbar[k] * cu(wF[:3])).sum()
            + (rho[k] * cu(wF[3])).sum())
    loss.backward()
    got = {f: p.grad.detach().cpu().numpy().astype(np.float64) for f, p in zip(FIELDS, params)}
    sc64 = orc.scene64(scene)
    args = (sc64, cam, t, d, 0, (0.0, 0.0, 0.0), pre, bins)
    # forward: one tile row
    row = GY // 2
    rmask = np.zeros(GX * GY, np.uint8)
    rmask[row * GX:(row + 1) * GX] = 1
    _, _, T64, D64 = orc.render_f64(*args, tile_mask=rmask, want_depth=True)
    ys = slice(row * 16, row * 16 + 16)
    clear = oracle_margin(pre, bins, cam, t, d, tiles=(row * GX, (row + 1) * GX))[ys] >= 1.0
    want = orc.normalized_depth_f64(D64, T64)[ys]
    hit = (want > 0) & clear
    rel = np.abs(dn[k].detach().cpu().numpy()[ys] - want)[hit] / want[hit]
    _, _, _, F = orc.render_f32(pre, bins, cam, t, d, want_feat=True, tiles=(row * GX, (row + 1) * GX))
    got_f = np.concatenate([vbar[k].detach().cpu().numpy(), rho[k].detach().cpu().numpy()[None]])[:, ys]
    ferr = float(np.abs(got_f - F[:, ys])[:, clear].max()) / max(1.0, float(np.abs(F[:, ys]).max()))
    print(f"[channels full size] row {row}: normalized depth max rel err {rel.max():.3g}, "
          f"velocity / staticness {ferr:.3g}")
    assert rel.max() <= 5e-5 and ferr <= 1e-5
    # backward on six tiles
    _, _, Tm, Dm = orc.render_f64(*args, tile_mask=m, want_depth=True)
    dD, dTn = orc.normalized_depth_bwd_f64(wD.astype(np.float64), Dm, Tm)
    zero = np.zeros((3, H, W))
    pD, _, tD = oracle_grads(orc, *args, zero, tile_mask=m, dD=dD)
    pT, _, tT = oracle_grads(orc, *args, zero, tile_mask=m, dT=dTn)
    pR, _, tR = oracle_grads(orc, *args, zero, tile_mask=m, dT=-wO.astype(np.float64), dF=wF.astype(np.float64))
    touched = np.zeros(scene["n"], bool)
    for f in FIELDS:
        touched |= (np.abs(pD[f]) + np.abs(pT[f]) + np.abs(pR[f])).reshape(-1, scene["n"]).max(axis=0) > 0
    assert touched.sum() > 100
    n = scene["n"]
    for f in FIELDS:
        ref = (pD[f] + pT[f] + pR[f]).reshape(-1, n)
        mag = sum(np.maximum(np.abs(pp[f]), 1e-2 * tt[f]) for pp, tt in ((pD, tD), (pT, tT), (pR, tR))).reshape(-1, n)
        g2 = got[f].reshape(-1, n)
        assert np.abs(g2[:, ~touched]).max() <= 1e-6 * max(np.abs(ref).max(), 1e-30), f
        worst, l2 = grad_tolerance_report(g2[:, touched], ref[:, touched], rel=1e-3, magnitude=mag[:, touched])
        plain, _ = grad_tolerance_report(g2[:, touched], ref[:, touched], rel=1e-3)
        print(f"[channels full size] {f}: worst/tol = {worst:.3g} (per-element bar on |g*| alone: {plain:.3g}), "
              f"l2 rel = {l2:.3g}")
        assert worst <= 1.0, f
