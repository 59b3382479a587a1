"""The fused Adam step and the opacity reset on the GPU against the FP64
oracle (itself pinned to torch.optim.Adam): three steps on a ragged
Gaussian count, then the moments carried through a densify pass."""
import numpy as np
import pytest

import gen
from helpers import FIELDS, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


LRS = {"mu": 4.8e-3, "scale": 5e-3, "rot": 1e-3, "sh0": 2.5e-3, "shN": 1.25e-4, "opacity": 0.005, "vel": 1e-3,
       "period": 0.0, "tau": 1e-3, "beta": 0.02}


def f32(x):
    return float(np.float32(x))


LRS32 = {k: f32(v) for k, v in LRS.items()}


@pytest.mark.parametrize("n", [1, 5003])
def test_adam_vs_fp64(orc, n):
    """Values within 2e-6 relative (plus 2e-6 of the rate), moments within
    1e-5 relative (plus 1e-6 of the row's largest) of the oracle after each
    of three steps; Gaussians with a
    zero gradient keep zero moments and their values bit for bit.  The
    configuration crosses the C ABI in FP32, so the oracle takes the same
    FP32-rounded rates, betas and eps (0.999 becomes 0.99900001287, which
    moves 1 - beta2 by 1.3e-5 relative)."""
    import paper_2311_18561_amd as pvg
    sc = gen.make_scene(n, 3, sh_degree=3)
    rng = np.random.default_rng(5)
    params = to_device(sc)
    opt = pvg.PVGAdam(params, LRS)
    ref = {k: (np.asarray(v, np.float64) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    rows = orc.optim.rows_of(ref)
    m = np.zeros((len(rows), n))
    v = np.zeros((len(rows), n))
    dead = np.zeros(n, bool)
    dead[::7] = True
    for t in range(1, 4):
        g = {f: (rng.standard_normal(np.shape(sc[f])) * 1e-2).astype(np.float32) for f in FIELDS}
        for f in FIELDS:
            g[f][..., dead] = 0.0
        opt.step(params, [torch.from_numpy(g[f]).cuda() for f in FIELDS])
        ref, m, v = orc.optim.adam_step(ref, {f: g[f].astype(np.float64) for f in FIELDS}, m, v, LRS32, t,
                                        beta1=f32(0.9), beta2=f32(0.999), eps=f32(1e-15))
        torch.cuda.synchronize()
        for f, p in zip(FIELDS, params):
            got = p.cpu().numpy().astype(np.float64)
            lr = max(LRS["sh0"], LRS["shN"]) if f == "sh" else LRS[f]
            err = np.abs(got - ref[f]) - (2e-6 * np.abs(ref[f]) + 2e-6 * lr)
            assert err.max() <= 0, (f, t, float(err.max()))
        mm = opt.moments.cpu().numpy().astype(np.float64)
        for got, want, name in ((mm[0], m, "m"), (mm[1], v, "v")):
            # m sums terms of either sign: near zero it is accurate relative to its row's scale
            row_scale = np.abs(want).max(axis=1, keepdims=True)
            err = np.abs(got - want) - (1e-5 * np.abs(want) + 1e-6 * row_scale)
            assert err.max() <= 0, (name, t, float(err.max()))
    assert not np.any(mm[:, :, dead])
    for f, p in zip(FIELDS, params):
        assert np.array_equal(p.cpu().numpy()[..., dead], np.asarray(sc[f])[..., dead]), f
    print(f"[adam n={n}] three steps within tolerance")


def test_opacity_reset_and_moments_through_densify(orc):
    import paper_2311_18561_amd as pvg
    n = 3000
    sc = gen.make_scene(n, 4, sh_degree=3)
    params = to_device(sc)
    opt = pvg.PVGAdam(params, LRS)
    rng = np.random.default_rng(6)
    opt.step(params, [torch.from_numpy((rng.standard_normal(np.shape(sc[f])) * 1e-2).astype(np.float32)).cuda()
                      for f in FIELDS])
    before = opt.moments.clone()
    opt.reset_opacity(params, 0.01)
    torch.cuda.synchronize()
    o = params[4].cpu().numpy()
    assert np.all(o <= np.float32(0.01))
    K = 16
    r_op = 3 + 3 + 4 + 3 * K
    mm = opt.moments.cpu().numpy()
    assert not np.any(mm[:, r_op])
    keep = np.ones(mm.shape[1], bool)
    keep[r_op] = False
    assert np.array_equal(mm[:, keep], before.cpu().numpy()[:, keep])
    # the moments ride through densify as carried rows
    acc = torch.from_numpy(rng.uniform(0, 5e-4, n).astype(np.float32)).cuda()
    cnt = torch.ones(n, device="cuda")
    noise = torch.randn((8, n), device="cuda")
    cfg = pvg.densify_config(30.0, min_opacity=0.0)
    new, rows = pvg.densify(params, acc, cnt, noise, cfg, opt.moments_rows())
    opt.set_moments_rows(rows)
    assert opt.moments.shape == (2, 17 + 3 * K, new[0].shape[1])
    opt.step(new, [torch.zeros_like(p) for p in new])  # runs on the new count


def test_adam_bench_shape(orc):
    """The benchmark's optimizer step: the 1M-Gaussian degree-3 scene with
    the default rates (r = 30), two steps, against the oracle with the bars
    of test_adam_vs_fp64."""
    import paper_2311_18561_amd as pvg
    sc = gen.make_config(2)["scene"]
    n = sc["n"]
    lrs = pvg.default_lrs(30.0)
    lrs32 = {k: f32(v) for k, v in lrs.items()}
    params = to_device(sc)
    opt = pvg.PVGAdam(params, lrs)
    ref = {k: (np.asarray(v, np.float64) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    rows = orc.optim.rows_of(ref)
    m = np.zeros((len(rows), n))
    v = np.zeros((len(rows), n))
    rng = np.random.default_rng(8)
    for t in (1, 2):
        g = {f: (rng.standard_normal(np.shape(sc[f])) * 1e-3).astype(np.float32) for f in FIELDS}
        opt.step(params, [torch.from_numpy(g[f]).cuda() for f in FIELDS])
        ref, m, v = orc.optim.adam_step(ref, {f: g[f].astype(np.float64) for f in FIELDS}, m, v, lrs32, t,
                                        beta1=f32(0.9), beta2=f32(0.999), eps=f32(1e-15))
    torch.cuda.synchronize()
    for f, p in zip(FIELDS, params):
        got = p.cpu().numpy().astype(np.float64)
        lr = max(lrs32["sh0"], lrs32["shN"]) if f == "sh" else lrs32[f]
        err = np.abs(got - ref[f]) - (2e-6 * np.abs(ref[f]) + 2e-6 * lr)
        assert err.max() <= 0, (f, float(err.max()))
    mm = opt.moments.cpu().numpy().astype(np.float64)
    for got, want, name in ((mm[0], m, "m"), (mm[1], v, "v")):
        row_scale = np.abs(want).max(axis=1, keepdims=True)
        err = np.abs(got - want) - (1e-5 * np.abs(want) + 1e-6 * row_scale)
        assert err.max() <= 0, (name, float(err.max()))
    print(f"[adam 1M] two steps within tolerance over {len(rows)} rows")


@pytest.mark.parametrize("res", [5, 1024])
def test_sky_cube_adam_vs_fp64(orc, res):
    """pvg_adam_dense on a [6,3,R,R] cube map (R = 5: a ragged count with
    the vector and tail paths; R = 1024: the training resolution of Sec. 4)
    against the FP64 oracle over three steps, with the bars of
    test_adam_vs_fp64; a face with a zero gradient keeps its texels."""
    import paper_2311_18561_amd as pvg
    rng = np.random.default_rng(9)
    cube0 = rng.uniform(0, 1, (6, 3, res, res)).astype(np.float32)
    cube = torch.from_numpy(cube0).cuda()
    opt = pvg.DenseAdam(cube, pvg.SKY_LR)
    lr = f32(pvg.SKY_LR)
    p, m, v = cube0.astype(np.float64), np.zeros(cube0.shape), np.zeros(cube0.shape)
    for t in range(1, 4):
        g = (rng.standard_normal(cube0.shape) * 1e-2).astype(np.float32)
        g[2] = 0.0
        opt.step(cube, torch.from_numpy(g).cuda())
        p, m, v = orc.optim.adam_dense(p, g.astype(np.float64), m, v, lr, t, beta1=f32(0.9), beta2=f32(0.999),
                                       eps=f32(1e-15))
        torch.cuda.synchronize()
        got = cube.cpu().numpy().astype(np.float64)
        err = np.abs(got - p) - (2e-6 * np.abs(p) + 2e-6 * lr)
        assert err.max() <= 0, (t, float(err.max()))
        for gm, want in ((opt.m, m), (opt.v, v)):
            e = np.abs(gm.cpu().numpy().astype(np.float64) - want) - (1e-5 * np.abs(want) + 1e-6 * np.abs(want).max())
            assert e.max() <= 0, (t, float(e.max()))
    assert np.array_equal(cube.cpu().numpy()[2], cube0[2])
    with pytest.raises(ValueError):
        opt.step(cube, torch.zeros((6, 3, res, res + 1), device="cuda"))
