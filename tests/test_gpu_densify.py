"""Adaptive control on the GPU (Sec. 3.3, Eq. (9)): the densify pass through
the C ABI against the oracle, and the view-space gradient statistics the
adjoint accumulates against the oracle's FP64 screen-space gradients.

The pass is bit-exact: every decision and every written value is the
oracle's FP32 arithmetic in the same order (correctly rounded division and
square root; the one exponential taken in FP64 and rounded once)."""
import numpy as np
import pytest

import gen
from helpers import FIELDS, oracle_margin, to_device, unambiguous

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CFG = dict(grad_threshold=1.7e-4, scene_radius=30.0, clone_scale=0.3, prune_scale=3.0, min_opacity=0.005,
           split_scale_decay=0.8, split_beta_decay=0.8)


def _inputs(n, seed, degree=3):
    sc = gen.make_scene(n, seed, sh_degree=degree) if n else None
    rng = np.random.default_rng(seed)
    if sc is not None:  # spread the means and sizes across every branch
        sc["mu"] = (sc["mu"] * rng.uniform(1, 40, n)).astype(np.float32)
        sc["scale"] = np.exp(rng.normal(-0.5, 1.5, (3, n))).astype(np.float32)
    acc = rng.uniform(0, 5e-4, n).astype(np.float32)
    cnt = rng.integers(0, 4, n).astype(np.float32)
    noise = rng.standard_normal((8, n)).astype(np.float32)
    extra = rng.standard_normal((5, n)).astype(np.float32)
    return sc, acc, cnt, noise, extra


def _gpu(sc, acc, cnt, noise, extra):
    import paper_2311_18561_amd as pvg
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    cfg = pvg.densify_config(CFG["scene_radius"], CFG["grad_threshold"], CFG["clone_scale"], CFG["prune_scale"],
                             CFG["min_opacity"], CFG["split_scale_decay"], CFG["split_beta_decay"])
    out, ex = pvg.densify(to_device(sc), cu(acc), cu(cnt), cu(noise), cfg, cu(extra))
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out], ex.cpu().numpy()


@pytest.mark.parametrize("n,seed", [(1, 1), (255, 2), (257, 3), (50_000, 4)])
def test_densify_bit_exact_vs_oracle(orc, n, seed):
    sc, acc, cnt, noise, extra = _inputs(n, seed)
    ref, ref_ex = orc.adaptive.densify(sc, acc, cnt, noise, CFG, extra)
    out, ex = _gpu(sc, acc, cnt, noise, extra)
    keeps = orc.adaptive.plan(sc, acc, cnt, noise, CFG)
    print(f"[n={n}] out {ref['n']}: kept {int(keeps[0].sum())}, clones {int(keeps[1].sum())}, "
          f"children {int(keeps[2].sum() + keeps[3].sum())}")
    assert out[0].shape[-1] == ref["n"]
    for f, o in zip(FIELDS, out):
        assert np.array_equal(o, ref[f]), f
    assert np.array_equal(ex, ref_ex)


def test_densify_branches_all_taken(orc):
    """The 50k case exercises every branch (so the bit-exact test above covers them)."""
    sc, acc, cnt, noise, _ = _inputs(50_000, 4)
    k0, k1, k2, k3 = orc.adaptive.plan(sc, acc, cnt, noise, CFG)
    split = (acc / np.maximum(cnt, 1) >= CFG["grad_threshold"]) & (cnt > 0) & ~k1 & ~k0
    assert k1.sum() > 100 and (k2 | k3).sum() > 100 and (~k0 & ~k1 & ~k2 & ~k3).sum() > 100
    assert split.sum() > 100


def test_densify_empty_and_all_pruned(orc):
    import paper_2311_18561_amd as pvg
    sc, acc, cnt, noise, extra = _inputs(300, 5)
    sc["opacity"][:] = 0.001  # below min_opacity: everything goes
    out, ex = _gpu(sc, acc, cnt, noise, extra)
    assert out[0].shape == (3, 0) and ex.shape == (5, 0)
    ref, _ = orc.adaptive.densify(sc, acc, cnt, noise, CFG)
    assert ref["n"] == 0
    e = torch.empty
    empty = [e((3, 0)), e((3, 0)), e((4, 0)), e((16, 3, 0)), e((0,)), e((3, 0)), e((0,)), e((0,)), e((0,))]
    params = [t.cuda() for t in empty]
    cfg = pvg.densify_config(30.0)
    out, _ = pvg.densify(params, e(0).cuda(), e(0).cuda(), e((8, 0)).cuda(), cfg)
    assert out[0].shape == (3, 0)


def test_densify_apply_rejects_wrong_output_size():
    import ctypes as C

    import paper_2311_18561_amd as pvg
    from paper_2311_18561_amd import _lib as L
    from paper_2311_18561_amd.render import _p, gaussians_struct
    sc, acc, cnt, noise, _ = _inputs(1000, 6)
    params = to_device(sc)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    cfg = pvg.densify_config(30.0)
    lib = L.load()
    size = C.c_size_t()
    L.check(lib.pvg_densify_tmp_bytes(1000, C.byref(size)))
    tmp = torch.empty(int(size.value), dtype=torch.uint8, device="cuda")
    g = gaussians_struct(params, 1000, 3)
    n_out = C.c_int64()
    nz = cu(noise)
    L.check(lib.pvg_densify_plan(C.byref(g), _p(cu(acc)), _p(cu(cnt)), _p(nz), C.byref(cfg), _p(tmp),
                                 int(tmp.numel()), C.byref(n_out), None))
    m = int(n_out.value) - 1  # one short
    out = [torch.empty((*p.shape[:-1], m), device="cuda") for p in params]
    go = gaussians_struct(out, m, 3)
    st = lib.pvg_densify_apply(C.byref(g), _p(nz), C.byref(cfg), _p(tmp), int(tmp.numel()), C.byref(go), 0, None,
                               None, None)
    assert st == -1  # PVG_ERR_INVALID, nothing written


@pytest.mark.parametrize("recompute", [False, True])
def test_view_space_statistics_vs_fp64(orc, recompute):
    """Two views (H(t) and the flow-translated render): each Gaussian's count
    is the number of views it is visible in (exact) and its sum of |(W/2
    dL/dx, H/2 dL/dy)| matches the FP64 adjoint's within 1e-3 relative (1e-2
    rms floor); statistics add up over calls."""
    import paper_2311_18561_amd as pvg
    cfg = gen.make_config(0)
    scene, cam, t = cfg["scene"], cfg["cameras"][0], cfg["t"]
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(12)
    dts = (0.0, 0.05)
    lists = [(pre, bins) for pre in [orc.preprocess_f32(scene, cam, t, d) for d in dts]
             for bins in [orc.bin_sort(pre, cam)]]
    # pixels whose skip or stop decisions are ambiguous carry no loss
    keep = np.stack([unambiguous(oracle_margin(pre, bins, cam, t, d, gradients=True))
                     for (pre, bins), d in zip(lists, dts)])
    w = (rng.standard_normal((2, 3, H, W)) * keep[:, None]).astype(np.float32)
    params = [p.requires_grad_(True) for p in to_device(scene)]
    n = scene["n"]
    acc = torch.zeros(n, device="cuda")
    cnt = torch.zeros(n, device="cuda")
    for rep in range(2):
        imgs = pvg.pvg_render_views(params, [(cam, t, d) for d in dts], recompute=recompute, stack=True,
                                    densify_stats=(acc, cnt))
        (imgs * torch.from_numpy(w).cuda()).sum().backward()
    g2ds, vis = [], []
    sc64 = orc.scene64(scene)
    for k, d in enumerate(dts):
        pre, bins = lists[k]
        _, g2d = orc.backward_f64(sc64, cam, t, d, 0, (0.0, 0.0, 0.0), pre, bins, w[k].astype(np.float64))
        g2ds.append(g2d)
        vis.append(pre["radius"] > 0)
    ref_acc, ref_cnt = orc.adaptive.view_space_stats(g2ds, vis, [(W, H)] * 2)
    got_cnt = cnt.cpu().numpy()
    assert np.array_equal(got_cnt, 2 * ref_cnt)
    got = acc.cpu().numpy().astype(np.float64)
    floor = 1e-2 * np.sqrt(np.mean((2 * ref_acc) ** 2))
    ratio = np.abs(got - 2 * ref_acc) / (1e-3 * np.maximum(2 * ref_acc, floor))
    print(f"[stats recompute={recompute}] worst/tol = {ratio.max():.3g}, visible (view 0) {int(vis[0].sum())}")
    assert ratio.max() <= 1.0


def test_densify_bench_shape_bit_exact(orc):
    """The benchmark's pass: the 1M-Gaussian driving-path scene, r = 30,
    threshold 1.7e-4, g = 0.01 r, b = 0.1 r, and the Adam moments of all 65
    parameter rows carried (130 rows: five row slices of the apply grid);
    bit-exact against the oracle."""
    import paper_2311_18561_amd as pvg
    sc = gen.make_config(2)["scene"]
    n = sc["n"]
    rng = np.random.default_rng(21)
    acc = rng.uniform(0, 4e-4, n).astype(np.float32)
    cnt = rng.integers(0, 7, n).astype(np.float32)
    noise = rng.standard_normal((8, n)).astype(np.float32)
    extra = rng.standard_normal((130, n)).astype(np.float32)
    cfg = dict(grad_threshold=1.7e-4, scene_radius=30.0, clone_scale=0.3, prune_scale=3.0, min_opacity=0.0,
               split_scale_decay=0.8, split_beta_decay=1.0)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    out, ex = pvg.densify(to_device(sc), cu(acc), cu(cnt), cu(noise), pvg.densify_config(30.0), cu(extra))
    ref, ref_ex = orc.adaptive.densify(sc, acc, cnt, noise, cfg, extra)
    keeps = orc.adaptive.plan(sc, acc, cnt, noise, cfg)
    print(f"[densify 1M] out {ref['n']}: clones {int(keeps[1].sum())}, children {int(keeps[2].sum() + keeps[3].sum())}, "
          f"pruned {int(n - keeps[0].sum() - (keeps[2] | keeps[3]).sum())}")
    assert out[0].shape[-1] == ref["n"]
    for f, o in zip(FIELDS, out):
        assert np.array_equal(o.cpu().numpy(), ref[f]), f
    assert np.array_equal(ex.cpu().numpy(), ref_ex)
