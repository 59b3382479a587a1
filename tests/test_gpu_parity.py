"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: bit-exact per-Gaussian discrete structure (radius, tile counts, depth
keys, 2D mean and conic), bit-exact sorted instances and ranges; images within
1e-4 absolute of the FP32 oracle; gradients within 1e-3 relative of the FP64
oracle (per element, relative to max(|g*|, 1e-2 rms(g*)) of that tensor, and
at least 1e-2 of the magnitude of the element's terms, since an FP32 sum is
accurate relative to its terms, not to a total that cancels).
The compositing walk's skip and stop decisions are discrete: where the
oracle's exact value sits within rounding of a threshold (its decision
margin below 1) either branch is a correct FP32 render, so images are held to
the bar at the other pixels, last contributors may differ only there, and
the losses whose gradients are compared give those pixels zero weight.

The product path lists a Gaussian only in tiles it can reach (tile culling);
its lists are checked to be the rectangle lists minus entries that every pixel
skips, and its images against the rectangle-list path bit for bit.
"""
import numpy as np
import pytest

import gen
from helpers import (FIELDS, check_culled_lists, geom_as_oracle_pre, gpu_forward, grad_tolerance_report,
                     image_parity, last_contributor_ids, oracle_grads, oracle_margin, to_device, unambiguous)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cases():
    return {
        "cfg0": lambda: (gen.make_config(0)["scene"], gen.make_config(0)["cameras"][0], 0.5, 0.0, 0, (0, 0, 0)),
        "ragged_dt": lambda: (gen.make_scene(3000, 21, sh_degree=2), gen.yaw_camera(200, 136, 15.0, (0.5, 0, -1)),
                              0.31, 0.05, 0, (0.2, 0.1, 0.0)),
        "cfg1_20k_raw_v": lambda: (gen.make_config(1, n=20_000)["scene"], gen.make_config(1, n=20_000)["cameras"][0],
                                   0.5, 0.05, 1, (0, 0, 0)),
    }


CASES = _cases()


@pytest.fixture(scope="module", params=list(CASES))
def case(request, orc):
    scene, cam, t, dt, mode, bg = CASES[request.param]()
    g = gpu_forward(scene, cam, t, dt, mode, bg)
    gr = gpu_forward(scene, cam, t, dt, mode, bg, params=g["_params"], tile_cull=False)
    o = orc.render(scene, cam, t, dt, mode, bg)
    return request.param, scene, cam, (t, dt, mode, bg), g, o, gr


def test_preprocess_bit_exact(case):
    name, scene, cam, fr, g, o, gr = case
    pre = o["pre"]
    print(f"[{name}] visible gpu={int((g['radius'] > 0).sum())} oracle={int((pre['radius'] > 0).sum())}")
    assert np.array_equal(g["radius"], pre["radius"])
    assert np.array_equal(g["tiles"], pre["tiles"])
    vis = pre["radius"] > 0
    assert vis.sum() > 0
    assert np.array_equal(g["depth"][vis].view(np.uint32), pre["depth"][vis].view(np.uint32))
    assert np.array_equal(g["xy"][vis], pre["xy"][vis])
    assert np.array_equal(g["conic_op"][vis], pre["conic_op"][vis])
    # colour: a different (but equal on the sphere) polynomial form of the SH basis
    np.testing.assert_allclose(g["rgb"][vis], pre["rgb"][vis], atol=2e-6, rtol=0)


def test_bin_sort_exact(case, orc):
    name, scene, cam, fr, g, o, gr = case
    b = o["bins"]
    assert gr["M"] == b["M"] and gr["L"] == b["M"]
    assert np.array_equal(gr["vals"], b["inst_gauss"])
    assert np.array_equal(gr["keys"], b["inst_tile"])
    assert np.array_equal(gr["ranges"], b["ranges"])
    # same check with the GPU's own record fed to the oracle's sort (structure injection)
    bins2 = orc.bin_sort(geom_as_oracle_pre(gr, cam), cam)
    assert np.array_equal(gr["vals"], bins2["inst_gauss"])


def test_culled_lists_valid(case):
    name, scene, cam, fr, g, o, gr = case
    b = o["bins"]
    assert g["M"] == g["L"] and g["L"] <= b["M"]
    dropped = check_culled_lists(g["keys"], g["vals"], g["ranges"], b["inst_tile"], b["inst_gauss"], o["pre"], cam,
                                 scene["n"])
    print(f"[{name}] rectangle instances {b['M']}, listed {g['L']}, removed {dropped}")
    assert dropped == b["M"] - g["L"]


def test_render_forward_parity(case):
    name, scene, cam, fr, g, o, gr = case
    margin = oracle_margin(o["pre"], o["bins"], cam, *fr)
    amb = margin < 1.0
    ids_orc = last_contributor_ids(o["n_contrib"], o["bins"]["inst_gauss"], o["bins"]["ranges"], cam["width"])
    for label, x in (("culled", g), ("rect", gr)):
        err, excused = image_parity(x["img"], o["img"], margin)
        terr, _ = image_parity(x["final_T"], o["final_T"], margin)
        ids = last_contributor_ids(x["n_contrib"], x["vals"], x["ranges"], cam["width"])
        flips = ids != ids_orc
        print(f"[{name}/{label}] max |img - oracle| = {err:.3g}, max |T - oracle| = {terr:.3g} (unambiguous "
              f"pixels), ambiguous pixels {int(amb.sum())}, excused {excused}, last-contributor flips "
              f"{int(flips.sum())}")
        assert not np.any(flips & ~amb)
    assert np.array_equal(gr["n_contrib"][~amb], o["n_contrib"][~amb])
    # culling removes only entries every pixel skips: identical compositing
    assert np.array_equal(g["img"], gr["img"]) and np.array_equal(g["final_T"], gr["final_T"])


def test_forward_deterministic(case):
    name, scene, cam, fr, g, o, gr = case
    for tc, ref in ((True, g), (False, gr)):
        g2 = gpu_forward(scene, cam, *fr, params=g["_params"], tile_cull=tc)
        for k in ("img", "final_T", "n_contrib", "vals", "keys", "ranges", "xy", "conic_op", "rgb"):
            assert np.array_equal(ref[k], g2[k]), (tc, k)


def _backward_compare(orc, scene, cam, t, dt, mode, bg, seed=0, rel=1e-3, tile_cull=True):
    import paper_2311_18561_amd as pvg
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(seed)
    pre = orc.preprocess_f32(scene, cam, t, dt, mode, bg)
    bins = orc.bin_sort(pre, cam)
    keep = unambiguous(oracle_margin(pre, bins, cam, t, dt, mode, bg, gradients=True))
    w = rng.standard_normal((3, H, W)).astype(np.float32) * keep
    params = [p.requires_grad_(True) for p in to_device(scene)]
    img = pvg.pvg_render(params, cam, t, dt, mode, bg, tile_cull=tile_cull)
    (img * torch.from_numpy(w).cuda()).sum().backward()
    ref, _, terms = oracle_grads(orc, orc.scene64(scene), cam, t, dt, mode, bg, pre, bins, w.astype(np.float64))
    report = {}
    for f, p in zip(FIELDS, params):
        got = p.grad.detach().cpu().numpy().astype(np.float64)
        report[f] = grad_tolerance_report(got, ref[f], rel=rel, terms=terms[f])
        if report[f][0] > 0.5:  # describe the worst element
            r = ref[f].reshape(-1)
            gg = got.reshape(-1)
            floor = 1e-2 * np.sqrt(np.mean(r ** 2))
            j = int(np.argmax(np.abs(gg - r) / (rel * np.maximum(np.abs(r), floor))))
            print(f"  {f}[{j}]: got {gg[j]:.9g} ref {r[j]:.9g} floor {floor:.3g} (entry {j % scene['n']})")
    return report


@pytest.mark.parametrize("name,dt,mode", [("tiny", 0.0, 0), ("tiny_dt", 0.05, 0), ("tiny_dt_raw", 0.05, 1)])
def test_backward_tiny_vs_fp64(orc, name, dt, mode):
    scene = gen.make_scene(60, 7, sh_degree=3)
    cam = gen.yaw_camera(80, 56, 10.0, (0.2, 0.1, -0.5))
    rep = _backward_compare(orc, scene, cam, 0.45, dt, mode, (0.1, 0.2, 0.3))
    for f, (worst, l2) in rep.items():
        print(f"[{name}] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f


@pytest.mark.parametrize("tile_cull", [True, False])
def test_backward_cfg0_vs_fp64(orc, tile_cull):
    cfg = gen.make_config(0)
    rep = _backward_compare(orc, cfg["scene"], cfg["cameras"][0], cfg["t"], 0.05, 0, (0, 0, 0), tile_cull=tile_cull)
    for f, (worst, l2) in rep.items():
        print(f"[cfg0 cull={tile_cull}] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f


@pytest.mark.parametrize("tile_cull", [True, False])
def test_backward_cfg1_20k_vs_fp64(orc, tile_cull):
    """Both list forms on 20k Gaussians at 960x640 (many tiles per splat, so
    the gather's whole-wave path runs) against the FP64 adjoint."""
    cfg = gen.make_config(1, n=20_000)
    rep = _backward_compare(orc, cfg["scene"], cfg["cameras"][0], cfg["t"], 0.05, 0, (0, 0, 0), seed=5,
                            tile_cull=tile_cull)
    for f, (worst, l2) in rep.items():
        print(f"[cfg1-20k cull={tile_cull}] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f


def test_backward_cfg1_subset_vs_fp64(orc):
    """The 500-Gaussian subset of the 960x640 degree-3 workload."""
    cfg = gen.make_config(1, n=20_000)
    cam = cfg["cameras"][0]
    pre = orc.preprocess_f32(cfg["scene"], cam, cfg["t"])
    rng = np.random.default_rng(2)
    idx = np.sort(rng.choice(np.nonzero(pre["tiles"] > 0)[0], 500, replace=False))
    sub = gen.subset_scene(cfg["scene"], idx)
    rep = _backward_compare(orc, sub, cam, cfg["t"], 0.05, 0, (0, 0, 0), seed=4)
    for f, (worst, l2) in rep.items():
        print(f"[cfg1-500] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f


def test_recompute_and_kept_lists_agree(orc):
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(0)
    cam = cfg["cameras"][0]
    grads = []
    for recompute in (True, False):
        params = [p.requires_grad_(True) for p in to_device(cfg["scene"])]
        img = pvg.pvg_render(params, cam, cfg["t"], 0.05, 0, (0, 0, 0), recompute)
        (img.square().sum()).backward()
        grads.append([p.grad.detach().cpu().numpy() for p in params])
    for a, b in zip(*grads):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * (1 + np.abs(b).max()))


@pytest.mark.parametrize("nviews", [1, 2, 3, 4, 7])
def test_render_views_any_view_count(nviews):
    """render_views with fewer, as many and more views than concurrent lanes
    (every chunking of the preprocess): each image equals the single-view
    render bit for bit, also when the pool hands back memory that held other
    data, and the differentiable path agrees with it."""
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(1, n=20_000)
    params = to_device(cfg["scene"])
    views = [(gen.yaw_camera(320, 208, -24.0 + 8.0 * k, (0.0, 0.0, 0.0)), 0.3 + 0.05 * k, 0.05 * (k % 2))
             for k in range(nviews)]
    ref = [pvg.render(params, cam, t, dt)[0].clone() for cam, t, dt in views]
    for _ in range(2):
        junk = torch.full((64 << 20,), 7.5e30, device="cuda")  # freed, so the pool reuses it for records
        del junk
        got = pvg.render_views(params, views)
        for k, (img, *_rest) in enumerate(got):
            assert torch.equal(img, ref[k]), (nviews, k)
    with torch.no_grad():
        stacked = pvg.pvg_render_views(params, views, stack=True)
    for k in range(nviews):
        assert torch.equal(stacked[k], ref[k]), (nviews, k)


def test_preprocess_views_equals_single_view_preprocess():
    """pvg_preprocess_views writes, for each view, exactly the record
    pvg_preprocess writes (ten views: two passes of up to eight; several
    cameras, times, flow offsets and both advection modes)."""
    import importlib
    R = importlib.import_module("paper_2311_18561_amd.render")
    cfg = gen.make_config(1, n=20_000)
    params = to_device(cfg["scene"])
    n, degree = cfg["scene"]["n"], cfg["scene"]["sh_degree"]
    cams, frames = [], []
    for k in range(10):
        cam = gen.yaw_camera(320 - 16 * (k % 3), 208, -30.0 + 6.0 * k, (0.0, 0.0, 0.5 * k))
        cams.append(R.camera_struct(cam))
        frames.append(R.frame_struct(0.1 * k, 0.05 * (k % 2), k % 2, (0.0, 0.0, 0.0)))
    multi = R.preprocess_views(params, n, degree, cams, frames)
    for k, (c, f) in enumerate(zip(cams, frames)):
        ref = R.preprocess(params, n, degree, c, f)
        for a, b in zip(multi[k].tensors(), ref.tensors()):
            assert torch.equal(a, b), k
        assert int((ref.radius > 0).sum()) > 100, k


@pytest.mark.parametrize("recompute", [True, False])
def test_multi_view_render_matches_single_views(orc, recompute):
    """pvg_render_views: each image equals the single-view render bit for bit;
    the gradients (the views' screen-space gradients taken through one
    per-Gaussian chain in the kernels) and the sum of the single-view
    gradients both match the FP64 oracle summed over the views, each element
    within 1e-3 of the sum over the views of max(|g*|, 1e-2 of its terms);
    a view that outgrows the cached capacity is redone."""
    import importlib
    import paper_2311_18561_amd as pvg
    R = importlib.import_module("paper_2311_18561_amd.render")
    cfg = gen.make_config(1, n=20_000)
    cams = [gen.yaw_camera(320, 208, yaw, (0.0, 0.0, 0.0)) for yaw in (-20.0, 0.0, 20.0)]
    views = [(cam, 0.4, d) for cam in cams for d in (0.0, 0.05)]
    sc64 = orc.scene64(cfg["scene"])
    ramp = np.linspace(-1, 1, 3 * 208 * 320).reshape(3, 208, 320)
    ref = {f: np.zeros_like(sc64[f]) for f in FIELDS}
    mag = {f: np.zeros_like(sc64[f]) for f in FIELDS}
    wn = []
    for k, (cam, t, d) in enumerate(views):
        pre = orc.preprocess_f32(cfg["scene"], cam, t, d)
        bins = orc.bin_sort(pre, cam)
        keep = unambiguous(oracle_margin(pre, bins, cam, t, d, gradients=True))
        wk = (ramp * (k + 1) * keep).astype(np.float32)
        wn.append(wk)
        part, _, terms = oracle_grads(orc, sc64, cam, t, d, 0, (0, 0, 0), pre, bins, wk.astype(np.float64))
        for f in FIELDS:
            ref[f] += part[f]
            mag[f] += np.maximum(np.abs(part[f]), 1e-2 * terms[f])
    w = [torch.from_numpy(x).cuda() for x in wn]
    ref_imgs, ref_grads = [], None
    params = [p.requires_grad_(True) for p in to_device(cfg["scene"])]
    for k, (cam, t, d) in enumerate(views):
        img = pvg.pvg_render(params, cam, t, d)
        ref_imgs.append(img.detach().clone())
        (img * w[k]).sum().backward()
    ref_grads = [p.grad.detach().clone() for p in params]
    for shrink in (False, True):
        if shrink:  # force an overflow of the cached capacity on every view
            for key in list(R._capacity_hint):
                R._capacity_hint[key] = 64
        params = [p.requires_grad_(True) for p in to_device(cfg["scene"])]
        imgs = pvg.pvg_render_views(params, views, recompute=recompute)
        sum((img * w[k]).sum() for k, img in enumerate(imgs)).backward()
        for a, b in zip(imgs, ref_imgs):
            assert torch.equal(a.detach(), b)
        for f, p, g in zip(FIELDS, params, ref_grads):
            for label, got in (("multi-view", p.grad), ("single views", g)):
                worst, l2 = grad_tolerance_report(got.cpu().numpy(), ref[f], magnitude=mag[f])
                assert worst <= 1.0, (label, shrink, f, worst)
        # the same views as one stacked [V,3,H,W] output
        for p in params:
            p.grad = None
        stacked = pvg.pvg_render_views(params, views, recompute=recompute, stack=True)
        assert stacked.shape == (6, 3, 208, 320)
        (stacked * torch.stack(w)).sum().backward()
        for k, b in enumerate(ref_imgs):
            assert torch.equal(stacked[k].detach(), b)
        for f, p in zip(FIELDS, params):
            worst, l2 = grad_tolerance_report(p.grad.cpu().numpy(), ref[f], magnitude=mag[f])
            assert worst <= 1.0, ("stacked", shrink, f, worst)


def test_edge_cases(orc):
    import paper_2311_18561_amd as pvg
    cam = gen.make_camera(72, 40)  # ragged 4.5 x 2.5 tiles
    # empty scene
    empty = gen.make_scene(0, 0)
    img, T, nc, geom, bins = pvg.render(to_device(empty), cam, 0.5, bg=(0.3, 0.2, 0.1))
    assert bins.num_instances == 0
    assert torch.all(img[0] == 0.3) and torch.all(T == 1) and torch.all(nc == 0)
    # everything behind the camera
    sc = gen.make_scene(500, 3)
    sc["mu"][2] = -np.abs(sc["mu"][2])
    img, T, nc, geom, bins = pvg.render(to_device(sc), cam, 0.5)
    assert bins.num_instances == 0 and torch.all(img == 0)
    # one Gaussian covering every tile, and a long single-tile list (> many batches)
    n = 3000
    mus = np.zeros((3, n), np.float32)
    mus[2] = np.linspace(2.0, 9.0, n)
    big = {"n": n, "sh_degree": 0, "mu": mus, "scale": np.full((3, n), 0.004, np.float32),
           "rot": np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, n)),
           "sh": np.full((1, 3, n), 0.3, np.float32), "opacity": np.full(n, 0.02, np.float32),
           "vel": np.zeros((3, n), np.float32), "period": np.ones(n, np.float32),
           "tau": np.full(n, 0.5, np.float32), "beta": np.full(n, 1e8, np.float32)}
    big["scale"][:, 0] = 3.0
    o = orc.render(big, cam, 0.5)
    gr = gpu_forward(big, cam, 0.5, tile_cull=False)
    assert gr["M"] == o["bins"]["M"]
    assert np.array_equal(gr["vals"], o["bins"]["inst_gauss"])
    margin = oracle_margin(o["pre"], o["bins"], cam, 0.5)
    image_parity(gr["img"], o["img"], margin)
    assert np.array_equal(gr["n_contrib"][margin >= 1], o["n_contrib"][margin >= 1])
    g = gpu_forward(big, cam, 0.5, params=gr["_params"])
    check_culled_lists(g["keys"], g["vals"], g["ranges"], o["bins"]["inst_tile"], o["bins"]["inst_gauss"], o["pre"],
                       cam, n)
    assert np.array_equal(g["img"], gr["img"])


@pytest.mark.parametrize("tile_cull", [True, False])
def test_faint_scene_lists_nothing(tile_cull):
    """Visible Gaussians whose opacity is below 1/255: the culled lists are
    empty while the rectangle lists are not; both render the background and
    give zero gradients."""
    import paper_2311_18561_amd as pvg
    sc = gen.make_scene(400, 9)
    sc["opacity"][:] = np.float32(1e-3)
    cam = gen.make_camera(96, 64)
    params = [p.requires_grad_(True) for p in to_device(sc)]
    img, T, nc, geom, bins = pvg.render(params, cam, 0.5, bg=(0.2, 0.3, 0.4), tile_cull=tile_cull)
    assert bins.num_visible > 0
    assert (bins.num_instances == 0) == tile_cull
    assert torch.all(T == 1) and torch.all(nc == 0)
    img = pvg.pvg_render(params, cam, 0.5, bg=(0.2, 0.3, 0.4), tile_cull=tile_cull)
    img.sum().backward()
    for f, p in zip(FIELDS, params):
        assert torch.count_nonzero(p.grad) == 0, f


@pytest.mark.parametrize("tile_cull", [False, True])
def test_capacity_handling(tile_cull):
    import ctypes as C
    import paper_2311_18561_amd as pvg
    from paper_2311_18561_amd import _lib as L
    cfg = gen.make_config(0)
    cam = cfg["cameras"][0]
    params = to_device(cfg["scene"])
    img, T, nc, geom, bins = pvg.render(params, cam, 0.5, tile_cull=tile_cull)
    M = bins.num_instances
    c = pvg.camera_struct(cam)
    from paper_2311_18561_amd.render import Bins, _p, _stream_handle, workspace
    small = Bins(16, bins.ranges.shape[0], params[0].device, geom.n, tile_cull)
    ws = workspace(geom.n, cam["width"], cam["height"], 16)
    tmp = torch.empty(int(ws.bin_tmp_bytes), dtype=torch.uint8, device="cuda")
    bs = small.struct()
    st = L.load().pvg_bin_sort(C.byref(geom.struct()), C.byref(c), C.byref(bs), _p(tmp), int(ws.bin_tmp_bytes), 1,
                               _stream_handle())
    assert st == L.PVG_ERR_CAPACITY
    # the count that did not fit: the instances, or (culled) first the rectangle rows
    assert bs.num_instances == M if not tile_cull else bs.num_instances > 16
    # without the host count: overflow flag on the device, empty ranges, background image
    st = L.load().pvg_bin_sort(C.byref(geom.struct()), C.byref(c), C.byref(bs), _p(tmp), int(ws.bin_tmp_bytes), 0,
                               _stream_handle())
    assert st == 0
    torch.cuda.synchronize()
    cnt = small.counters.cpu().numpy().view(np.uint32)
    assert cnt[2] == 1 and cnt[0] == 0
    if not tile_cull:
        assert cnt[3] == M
    assert torch.all(small.ranges == 0)
    img2, _, _ = pvg.render_fwd(geom, small, c, pvg.frame_struct(0.5, bg=(0.5, 0.5, 0.5)))
    assert torch.all(img2 == 0.5)
    # the Python layer grows the capacity until it fits and reproduces the image
    img3, _, _, _, bins3 = pvg.render(params, cam, 0.5, tile_cull=tile_cull)
    assert bins3.num_instances == M and torch.equal(img3, img)


def test_config1_full_size(orc):
    """The 200k-Gaussian, 960x640, degree-3 workload at full size: forward
    against the FP32 oracle, L1-loss gradients against the FP64 oracle."""
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(1)
    cam, t = cfg["cameras"][0], cfg["t"]
    scene = cfg["scene"]
    g = gpu_forward(scene, cam, t)
    gr = gpu_forward(scene, cam, t, params=g["_params"], tile_cull=False)
    o = orc.render(scene, cam, t)
    assert gr["M"] == o["bins"]["M"] and g["M"] == g["L"] < gr["M"]
    assert np.array_equal(g["radius"], o["pre"]["radius"])
    assert np.array_equal(gr["vals"], o["bins"]["inst_gauss"])
    assert np.array_equal(gr["keys"], o["bins"]["inst_tile"])
    dropped = check_culled_lists(g["keys"], g["vals"], g["ranges"], o["bins"]["inst_tile"], o["bins"]["inst_gauss"],
                                 o["pre"], cam, scene["n"], sample=200_000)
    assert np.array_equal(g["img"], gr["img"])
    margin = oracle_margin(o["pre"], o["bins"], cam, t)
    amb = margin < 1.0
    err, excused = image_parity(g["img"], o["img"], margin)
    ids = last_contributor_ids(g["n_contrib"], g["vals"], g["ranges"], cam["width"])
    ids_orc = last_contributor_ids(o["n_contrib"], o["bins"]["inst_gauss"], o["bins"]["ranges"], cam["width"])
    flips = ids != ids_orc
    print(f"[cfg1] M={g['M']} listed={g['L']} (removed {dropped}) max |img - oracle| = {err:.3g} at unambiguous "
          f"pixels; ambiguous {int(amb.sum())}, excused {excused}, last-contributor flips {int(flips.sum())}")
    assert not np.any(flips & ~amb)
    # the L1 loss's gradient at the oracle's image, on the unambiguous pixels
    keep = unambiguous(oracle_margin(o["pre"], o["bins"], cam, t, gradients=True))
    dimg = (np.sign(o["img"].astype(np.float64) - cfg["targets"][0]) / (3 * 640 * 960) * keep).astype(np.float32)
    params = [p.requires_grad_(True) for p in to_device(scene)]
    img = pvg.pvg_render(params, cam, t)
    (img * torch.from_numpy(dimg).cuda()).sum().backward()
    dimg = dimg.astype(np.float64)
    ref, _, terms = oracle_grads(orc, orc.scene64(scene), cam, t, 0.0, 0, (0, 0, 0), o["pre"], o["bins"], dimg)
    for f, p in zip(FIELDS, params):
        worst, l2 = grad_tolerance_report(p.grad.detach().cpu().numpy(), ref[f], terms=terms[f])
        print(f"[cfg1] {f}: worst/tol = {worst:.3g}, l2 rel = {l2:.3g}")
        assert worst <= 1.0, f
