"""Pins of the adaptive-control oracle (Sec. 3.3, Eq. (9); the split rules of
the appendix's implementation details): Eq. (9)'s values and limits, hand
cases of every branch (keep, clone, split, prune, the position-aware
thresholds far from the centre), the split child's mean against scipy's
rotation in FP64, the output order and the carried rows."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import adaptive as ad

CFG = dict(grad_threshold=1.7e-4, scene_radius=30.0, clone_scale=0.3, prune_scale=3.0, min_opacity=0.0,
           split_scale_decay=0.8, split_beta_decay=1.0)


def scene(mus, scales, rot=None, vel=None, beta=None, period=None, tau=None, opacity=None, degree=0):
    mus = np.asarray(mus, np.float32).T
    n = mus.shape[1]
    K = (degree + 1) ** 2
    rng = np.random.default_rng(0)
    return {"n": n, "sh_degree": degree, "mu": mus,
            "scale": np.asarray(scales, np.float32).T if np.ndim(scales) == 2 else np.tile(
                np.asarray(scales, np.float32)[None], (3, 1)),
            "rot": np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)) if rot is None
            else np.asarray(rot, np.float32).T,
            "sh": rng.standard_normal((K, 3, n)).astype(np.float32),
            "opacity": np.full(n, 0.5, np.float32) if opacity is None else np.asarray(opacity, np.float32),
            "vel": np.zeros((3, n), np.float32) if vel is None else np.asarray(vel, np.float32).T,
            "period": np.full(n, 2.0, np.float32) if period is None else np.asarray(period, np.float32),
            "tau": np.full(n, 0.4, np.float32) if tau is None else np.asarray(tau, np.float32),
            "beta": np.full(n, 0.3, np.float32) if beta is None else np.asarray(beta, np.float32)}


def test_gamma_values_and_limits():
    """Eq. (9): 1 for |mu| < 2r; |mu| / r - 1 beyond; continuous at 2r (both
    pieces give 1); 2 at 3r; invariant under scaling mu and r together."""
    r = 30.0
    mu = np.array([[0.0, 10.0, 59.9, 60.0, 90.0, 300.0], [0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 0]], np.float32)
    g = ad.gamma(mu, r)
    assert g[0] == 1.0 and g[1] == 1.0 and g[2] == 1.0
    assert g[3] == 1.0 and g[4] == 2.0 and g[5] == 9.0
    d = np.array([[3.0], [4.0], [12.0]], np.float32)  # |d| = 13
    for k in (0.5, 5.0, 10.0):
        np.testing.assert_allclose(ad.gamma(d * np.float32(k), 2.0 * k), ad.gamma(d, 2.0), rtol=1e-6)
    xs = np.linspace(0, 500, 2001, dtype=np.float32)
    gs = ad.gamma(np.stack([xs, 0 * xs, 0 * xs]), r)
    assert np.all(np.diff(gs) >= 0)


def _run(sc, grad, count=1.0, noise=None, cfg=CFG, extra=None):
    n = sc["n"]
    acc = np.full(n, grad * count, np.float32)
    cnt = np.full(n, count, np.float32)
    noise = np.zeros((8, n), np.float32) if noise is None else np.asarray(noise, np.float32)
    return ad.densify(sc, acc, cnt, noise, cfg, extra)


def test_low_gradient_keeps_everything_unchanged():
    sc = scene([[1.0, 2.0, 3.0], [4.0, 0.0, 1.0]], [0.1, 0.2])
    out, _ = _run(sc, 1e-5)
    assert out["n"] == 2
    for f in ad.ROWS:
        assert np.array_equal(out[f], sc[f]), f
    assert np.array_equal(out["sh"], sc["sh"])


def test_zero_count_never_densifies():
    sc = scene([[1.0, 2.0, 3.0]], [0.1])
    out, _ = _run(sc, 1.0, count=0.0)
    assert out["n"] == 1


def test_small_high_gradient_gaussian_is_cloned():
    """max(s) <= g gamma: the original and an identical copy."""
    sc = scene([[1.0, 2.0, 3.0]], [0.2])
    out, _ = _run(sc, 1e-3)
    assert out["n"] == 2
    for f in ad.ROWS:
        assert np.array_equal(out[f][..., 0], out[f][..., 1]) and np.array_equal(out[f][..., 0], sc[f][..., 0])


def test_large_high_gradient_gaussian_is_split():
    """max(s) > g gamma: two children with scale 0.8 s, tau + beta eps3 and
    mean mu + R(q) (s * eps); the mean checked against scipy's rotation of
    the normalised quaternion in FP64."""
    rng = np.random.default_rng(3)
    q = np.array([0.9, -0.3, 0.2, 0.4])
    s = np.array([[0.5, 0.8, 1.2]])
    sc = scene([[1.0, -2.0, 5.0]], s, rot=[q])
    eps = rng.standard_normal((8, 1)).astype(np.float32)
    out, _ = _run(sc, 1e-3, noise=eps)
    assert out["n"] == 2
    rot = Rotation.from_quat([q[1], q[2], q[3], q[0]])  # scipy takes (x, y, z, w)
    for k in range(2):
        want = np.array([1.0, -2.0, 5.0]) + rot.apply(s[0] * eps[4 * k:4 * k + 3, 0].astype(np.float64))
        np.testing.assert_allclose(out["mu"][:, k], want, rtol=0, atol=2e-6)
        np.testing.assert_array_equal(out["scale"][:, k], np.float32(0.8) * sc["scale"][:, 0])
        assert out["tau"][k] == np.float32(0.4) + np.float32(0.3) * eps[4 * k + 3, 0]
        assert out["beta"][k] == sc["beta"][0]
        for f in ("rot", "vel", "opacity", "period"):
            assert np.array_equal(out[f][..., k], sc[f][..., 0])


def test_split_moves_along_the_mean_velocity():
    """eps = 0 for the position, eps3 = 1: the child moves by beta v exp(-beta / (2 l)) (Eq. (10))."""
    v = np.array([2.0, -1.0, 0.5])
    sc = scene([[0.0, 0.0, 10.0]], [1.0], vel=[v], beta=[0.3], period=[1.5])
    eps = np.zeros((8, 1), np.float32)
    eps[3] = 1.0
    eps[7] = -2.0
    out, _ = _run(sc, 1e-3, noise=eps)
    vb = v * np.exp(-0.3 / (2 * 1.5))
    np.testing.assert_allclose(out["mu"][:, 0], np.array([0, 0, 10.0]) + 0.3 * vb, rtol=1e-6)
    np.testing.assert_allclose(out["mu"][:, 1], np.array([0, 0, 10.0]) - 0.6 * vb, rtol=1e-6)
    np.testing.assert_allclose(out["tau"], [0.4 + 0.3, 0.4 - 0.6], rtol=1e-6)


def test_beta_decay_in_split():
    sc = scene([[0.0, 0.0, 10.0]], [1.0])
    cfg = dict(CFG, split_beta_decay=0.8)
    out, _ = _run(sc, 1e-3, cfg=cfg)
    assert np.all(out["beta"] == np.float32(0.8) * np.float32(0.3))


def test_prune_by_size_and_opacity():
    """max(s) > b gamma is pruned; o < min_opacity is pruned; a split child
    is pruned by its own (shrunk) scale."""
    sc = scene([[0.0, 0.0, 5.0], [0.0, 0.0, 6.0], [0.0, 0.0, 7.0]], [3.5, 0.1, 3.5],
               opacity=[0.5, 0.001, 0.5])
    out, _ = _run(sc, 1e-5, cfg=dict(CFG, min_opacity=0.005))
    # no densification: the first is too big, the second too faint, the third too big as well
    assert out["n"] == 0
    # 3.5 * 0.8 = 2.8 <= b = 3: split children of the big ones survive
    out, _ = _run(sc, 1e-3, cfg=dict(CFG, min_opacity=0.005))
    assert out["n"] == 4 and np.allclose(out["scale"], 2.8)


def test_position_aware_thresholds_far_from_centre():
    """The same Gaussian (max s = 1) near the centre is split and far away
    (|mu| = 300 = 10 r, gamma = 9) cloned; a max s = 10 Gaussian is pruned
    near and kept far (b gamma = 27)."""
    near, far = [0.0, 0.0, 5.0], [0.0, 0.0, 300.0]
    out, _ = _run(scene([near], [1.0]), 1e-3)
    assert out["n"] == 2 and np.all(out["scale"] == np.float32(0.8))
    out, _ = _run(scene([far], [1.0]), 1e-3, cfg=dict(CFG, clone_scale=0.3))
    assert out["n"] == 2 and np.all(out["scale"] == 1.0)  # 1 <= 0.3 * 9: cloned
    assert ad.gamma(np.array([[0.0], [0.0], [300.0]], np.float32), 30.0)[0] == 9.0
    out, _ = _run(scene([near], [10.0]), 1e-5)
    assert out["n"] == 0
    out, _ = _run(scene([far], [10.0]), 1e-5)
    assert out["n"] == 1


def test_order_and_carried_rows():
    """Parents in index order; within one: original, clone, children; extra
    rows kept for originals, zero for new Gaussians."""
    sc = scene([[0.0, 0.0, 5.0], [0.0, 0.0, 6.0], [0.0, 0.0, 7.0]], [0.1, 1.0, 0.1])
    acc = np.array([1e-3, 1e-3, 1e-6], np.float32)
    cnt = np.ones(3, np.float32)
    extra = np.arange(6, dtype=np.float32).reshape(2, 3) + 1.0
    out, ex = ad.densify(sc, acc, cnt, np.zeros((8, 3), np.float32), CFG, extra)
    # parent 0 cloned (2), parent 1 split (2 children), parent 2 kept (1)
    assert out["n"] == 5
    np.testing.assert_array_equal(out["mu"][2], [5.0, 5.0, 6.0, 6.0, 7.0])
    np.testing.assert_array_equal(ex, [[1.0, 0.0, 0.0, 0.0, 3.0], [4.0, 0.0, 0.0, 0.0, 6.0]])


@pytest.mark.parametrize("n", [0, 1, 300])
def test_plan_counts_match_the_pass(n):
    rng = np.random.default_rng(n)
    sc = scene(rng.uniform(-100, 100, (n, 3)), np.exp(rng.normal(-1, 1, (n, 3))),
               rot=rng.standard_normal((n, 4)), vel=rng.normal(0, 1, (n, 3))) if n else scene(
        np.zeros((0, 3)), np.zeros((0, 3)))
    acc = rng.uniform(0, 4e-4, n).astype(np.float32)
    cnt = rng.integers(0, 4, n).astype(np.float32)
    noise = rng.standard_normal((8, n)).astype(np.float32)
    keeps = ad.plan(sc, acc, cnt, noise, CFG)
    out, _ = ad.densify(sc, acc, cnt, noise, CFG)
    assert out["n"] == int(sum(k.sum() for k in keeps))
    assert not np.any(keeps[0] & (keeps[2] | keeps[3]))  # a split parent is replaced
    assert not np.any(keeps[1] & ~keeps[0])  # a clone survives with its original


def test_staticness_split_partition():
    """rho = beta / l >= threshold is static (a point exactly at the
    threshold included); the two parts partition the Gaussians and keep
    their order."""
    rng = np.random.default_rng(9)
    n = 200
    sc = scene(rng.uniform(-10, 10, (n, 3)), np.exp(rng.normal(-1, 0.5, (n, 3))), beta=rng.uniform(0.05, 2, n),
               period=rng.uniform(0.5, 3, n))
    sc["beta"][0], sc["period"][0] = 1.5, 1.5  # rho exactly 1
    st, dy = ad.split_by_staticness(sc, 1.0)
    rho = sc["beta"] / sc["period"]
    assert st["n"] + dy["n"] == n and st["n"] == int((rho >= 1.0).sum())
    assert st["mu"][0, 0] == sc["mu"][0, 0]  # the threshold point is static, first in order
    idx_s = np.nonzero(rho >= 1.0)[0]
    idx_d = np.nonzero(rho < 1.0)[0]
    np.testing.assert_array_equal(st["tau"], sc["tau"][idx_s])
    np.testing.assert_array_equal(dy["sh"], sc["sh"][..., idx_d])
    a, b = ad.split_by_staticness(sc, 1e9)
    assert a["n"] == 0 and b["n"] == n
