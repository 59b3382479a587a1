"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names the passage of the paper (Periodic Vibration Gaussian,
arXiv 2311.18561) whose consequence it checks: closed forms, limits stated in
the paper, invariants, special cases that reduce to library routines, brute
force on tiny inputs, and finite differences of the FP64 adjoint.
"""
import math

import numpy as np
import pytest
import scipy.special as sps
from scipy.spatial.transform import Rotation

import gen

TILE = 16


def one_scene(mus, scales, opac, sh0=None, vel=None, tau=None, beta=None, period=None, rot=None):
    """Scene of explicit isotropic Gaussians (degree-0 colour)."""
    mus = np.asarray(mus, np.float64).T
    n = mus.shape[1]
    s = np.asarray(scales, np.float64)
    sc = {"n": n, "sh_degree": 0,
          "mu": mus,
          "scale": np.tile(s[None, :], (3, 1)) if s.ndim == 1 else s,
          "rot": np.tile(np.array([[1.0], [0.0], [0.0], [0.0]]), (1, n)) if rot is None else np.asarray(rot).T,
          "sh": (np.zeros((1, 3, n)) if sh0 is None else np.asarray(sh0, np.float64).T[None]),
          "opacity": np.asarray(opac, np.float64),
          "vel": np.zeros((3, n)) if vel is None else np.asarray(vel, np.float64).T,
          "period": np.ones(n) if period is None else np.asarray(period, np.float64),
          "tau": np.full(n, 0.5) if tau is None else np.asarray(tau, np.float64),
          "beta": np.full(n, 1e8) if beta is None else np.asarray(beta, np.float64)}
    return {k: (np.ascontiguousarray(v, np.float32) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}


Y00 = 0.5 / math.sqrt(math.pi)


# ---------------------------------------------------------------- P1, P2
def test_single_isotropic_gaussian_closed_form(orc):
    """Sec. 3.1 Eqs. (2)-(3): one isotropic Gaussian on the optical axis.

    J at (0,0,z0) is diag(f/z0) so Sigma' = (f s / z0)^2 I; alpha is the
    opacity times the 2D Gaussian (+0.3 px^2 low-pass) at the pixel, the pixel
    value is alpha * colour on a black background."""
    cam = gen.make_camera(128, 96)  # fx = fy = 100, cx = 64, cy = 48
    z0, s, o, shc = 6.0, 0.09, 0.7, 0.8
    sc = one_scene([[0.0, 0.0, z0]], [s], [o], sh0=[[shc, -0.4, 0.1]])
    r = orc.render(sc, cam, 0.5)
    f = 100.0
    var = (f * np.float32(s) / z0) ** 2 + 0.3
    ys, xs = np.mgrid[0:96, 0:128].astype(np.float64)
    d2 = (xs - 63.5) ** 2 + (ys - 47.5) ** 2
    alpha = np.minimum(0.99, np.float32(o) * np.exp(-0.5 * d2 / var))
    col = np.maximum(0.0, Y00 * np.array([shc, -0.4, 0.1], np.float32) + 0.5)
    rad = math.ceil(3.0 * math.sqrt(var + math.sqrt(0.1)))
    assert r["pre"]["radius"][0] == rad
    x0, x1 = max(0, math.floor((63.5 - rad) / 16)), min(8, math.floor((63.5 + rad + 15) / 16))
    y0, y1 = max(0, math.floor((47.5 - rad) / 16)), min(6, math.floor((47.5 + rad + 15) / 16))
    assert list(r["pre"]["rect"][0]) == [x0, y0, x1, y1]
    assert r["bins"]["M"] == (x1 - x0) * (y1 - y0)
    inside = np.zeros((96, 128), bool)
    inside[y0 * 16:y1 * 16, x0 * 16:x1 * 16] = True
    used = inside & (alpha >= 1.0 / 255.0)
    for c in range(3):
        exp_c = np.where(used, alpha * col[c], 0.0)
        np.testing.assert_allclose(r["img"][c], exp_c, atol=2e-6, rtol=0)
    np.testing.assert_allclose(r["final_T"], np.where(used, 1 - alpha, 1.0), atol=2e-6)
    assert np.array_equal(r["n_contrib"], used.astype(np.int32))
    # the depth key is the camera-space z (Sec. 3.1, ordering by depth)
    assert r["pre"]["depth"][0] == np.float32(z0)


def test_two_coaxial_gaussians_blend_front_to_back(orc):
    """Sec. 3.1 Eq. (3): C = a1 c1 + (1 - a1) a2 c2 with the nearer one first,
    whatever the storage order."""
    cam = gen.make_camera(128, 96)
    # far one stored first
    sc = one_scene([[0.0, 0.0, 9.0], [0.0, 0.0, 4.0]], [0.2, 0.05], [0.6, 0.5],
                   sh0=[[1.0, 0.0, -1.0], [-1.0, 1.0, 0.5]])
    r = orc.render(sc, cam, 0.5)
    ys, xs = np.mgrid[0:96, 0:128].astype(np.float64)
    d2 = (xs - 63.5) ** 2 + (ys - 47.5) ** 2

    def a(z, s, o):
        var = (100.0 * np.float32(s) / z) ** 2 + 0.3
        return np.minimum(0.99, np.float32(o) * np.exp(-0.5 * d2 / var))

    a_far, a_near = a(9.0, 0.2, 0.6), a(4.0, 0.05, 0.5)
    c_far = np.maximum(0, Y00 * np.array([1.0, 0.0, -1.0]) + 0.5)
    c_near = np.maximum(0, Y00 * np.array([-1.0, 1.0, 0.5]) + 0.5)
    # pixels where both contribute (alpha >= 1/255) and both rectangles hold the tile
    both = (a_far >= 1 / 255) & (a_near >= 1 / 255)
    yy, xx = np.nonzero(both)
    sel = (yy // 16 >= 1) & (yy // 16 <= 4) & (xx // 16 >= 2) & (xx // 16 <= 5)
    yy, xx = yy[sel], xx[sel]
    for c in range(3):
        exp_c = a_near * c_near[c] + (1 - a_near) * a_far * c_far[c]
        np.testing.assert_allclose(r["img"][c][yy, xx], exp_c[yy, xx], atol=3e-6)
    # the list of the centre tile is (near, far) = (1, 0)
    GX = 8
    t = 2 * GX + 3
    lo, hi = r["bins"]["ranges"][t]
    assert list(r["bins"]["inst_gauss"][lo:hi]) == [1, 0]


def test_termination_before_transmittance_drops_below_threshold(orc):
    """Eq. (3) with early termination: ten coaxial Gaussians of alpha 0.8 at
    the centre pixel; T_k = 0.2^k, the sixth would take T below 1e-4, so five
    contribute and C = sum_{k<5} 0.2^k 0.8 c."""
    cam = gen.make_camera(128, 96)
    # alpha = o at the 2D mean; put the mean on pixel (64, 48): x_c = 0.5 z / f
    zs = np.linspace(3.0, 8.0, 10)
    mus = [[0.5 * z / 100.0, 0.5 * z / 100.0, z] for z in zs]
    sc = one_scene(mus, [0.05] * 10, [0.8] * 10, sh0=[[1.0, 1.0, 1.0]] * 10)
    r = orc.render(sc, cam, 0.5)
    c = Y00 + 0.5
    a = np.float32(0.8)
    expect = sum(0.2 ** k * 0.8 * c for k in range(5))
    assert r["n_contrib"][48, 64] == 5
    np.testing.assert_allclose(r["img"][:, 48, 64], expect, rtol=1e-5)
    np.testing.assert_allclose(r["final_T"][48, 64], (1 - a) ** 5, rtol=1e-5)


def test_skip_rules(orc):
    """Eq. (3): a pair whose alpha is below 1/255 does not contribute."""
    cam = gen.make_camera(128, 96)
    sc = one_scene([[0.0, 0.0, 5.0]], [0.1], [1.0 / 300.0], sh0=[[1.0, 1.0, 1.0]])
    r = orc.render(sc, cam, 0.5)
    assert r["bins"]["M"] > 0
    assert np.all(r["img"] == 0.0) and np.all(r["n_contrib"] == 0) and np.all(r["final_T"] == 1.0)


def test_background_term(orc):
    """Eq. (3) on a background: C + T_final * bg (constant sky stand-in)."""
    cfg = gen.make_config(0)
    cam = cfg["cameras"][0]
    bg = (0.25, 0.5, 0.75)
    a = orc.render(cfg["scene"], cam, cfg["t"])
    b = orc.render(cfg["scene"], cam, cfg["t"], bg=bg)
    for c in range(3):
        np.testing.assert_allclose(b["img"][c], a["img"][c] + a["final_T"] * bg[c], atol=1e-6)


# ---------------------------------------------------------------- P3 temporal model
def test_vibration_at_life_peak_and_zero_velocity():
    """Eq. (6): mu~(tau) = mu; v = 0 gives mu~ = mu at every t."""
    import oracle
    mu, v = np.array([1.0, -2.0, 3.0]), np.array([0.3, -0.1, 0.2])
    m, op = oracle.temporal_f64(mu, v, 0.7, 0.4, 0.2, 0.6, 0.4)
    assert np.array_equal(m, mu) and op == 0.6
    for t in (0.0, 0.13, 0.9):
        m, _ = oracle.temporal_f64(mu, np.zeros(3), 0.7, 0.4, 0.2, 0.6, t)
        assert np.array_equal(m, mu)


def test_velocity_is_derivative_at_life_peak():
    """Sec. 3.2: v = d mu~/dt at t = tau."""
    import oracle
    mu, v = np.array([1.0, -2.0, 3.0]), np.array([0.3, -0.1, 0.2])
    h = 1e-6
    p, _ = oracle.temporal_f64(mu, v, 0.7, 0.4, 0.2, 0.6, 0.4 + h)
    m, _ = oracle.temporal_f64(mu, v, 0.7, 0.4, 0.2, 0.6, 0.4 - h)
    np.testing.assert_allclose((p - m) / (2 * h), v, rtol=1e-8)


def test_period_mean_is_the_mean_position():
    """Sec. 3.2: E[mu~(t)] = mu over any interval whose length is a multiple of l."""
    import oracle
    mu, v, l, tau = np.array([1.0, -2.0, 3.0]), np.array([0.3, -0.1, 0.2]), 0.7, 0.4
    for start, periods in ((0.0, 1), (0.31, 2), (-1.7, 3)):
        ts = start + (np.arange(4000) + 0.5) / 4000 * periods * l
        mean = np.mean([oracle.temporal_f64(mu, v, l, tau, 0.2, 0.6, t)[0] for t in ts], axis=0)
        np.testing.assert_allclose(mean, mu, atol=1e-9)


def test_limits_of_cycle_length():
    """Table 7 dynamics variants: l -> inf gives the linear model mu + v(t - tau)
    (error O(l^-2)); l -> 0 stays within l|v|/(2pi) of mu (constant model)."""
    import oracle
    mu, v, tau, t = np.array([1.0, -2.0, 3.0]), np.array([0.3, -0.1, 0.2]), 0.4, 0.9
    for l in (1e2, 1e3):
        m, _ = oracle.temporal_f64(mu, v, l, tau, 0.2, 0.6, t)
        err = np.abs(m - (mu + v * (t - tau))).max()
        bound = (2 * math.pi) ** 2 * abs(t - tau) ** 3 / (6 * l * l) * np.abs(v).max()
        assert err <= bound * 1.01
    l = 1e-4
    m, _ = oracle.temporal_f64(mu, v, l, tau, 0.2, 0.6, t)
    assert np.all(np.abs(m - mu) <= l * np.abs(v) / (2 * math.pi) * (1 + 1e-9))


def test_opacity_decay():
    """Eq. (7): o~(tau) = o; o~(tau + beta) = o e^{-1/2}; beta -> inf keeps o."""
    import oracle
    mu, v = np.zeros(3), np.zeros(3)
    _, op = oracle.temporal_f64(mu, v, 1.0, 0.3, 0.25, 0.8, 0.55)
    assert op == pytest.approx(0.8 * math.exp(-0.5), rel=1e-14)
    _, op = oracle.temporal_f64(mu, v, 1.0, 0.3, 1e8, 0.8, 0.9)
    assert op == 0.8


def test_average_velocity_limits_and_flow_translation():
    """Eqs. (10), (12): mu^ = mu~(t) + v_bar dt with v_bar = v exp(-rho/2),
    rho = beta/l; v_bar -> 0 as rho -> inf and -> v as rho -> 0."""
    import oracle
    mu, v, l, tau, t, dt = np.array([1.0, 2.0, 3.0]), np.array([0.3, -0.1, 0.2]), 0.8, 0.3, 0.6, 0.05
    base, _ = oracle.temporal_f64(mu, v, l, tau, 0.4, 0.6, t)
    adv, _ = oracle.temporal_f64(mu, v, l, tau, 0.4, 0.6, t, dt, 0)
    np.testing.assert_allclose((adv - base) / dt, v * math.exp(-0.5 * 0.4 / l), rtol=1e-12)
    big, _ = oracle.temporal_f64(mu, v, l, tau, 0.8e6, 0.6, t, dt, 0)
    b2, _ = oracle.temporal_f64(mu, v, l, tau, 0.8e6, 0.6, t)
    np.testing.assert_allclose(big, b2, atol=0)
    small, _ = oracle.temporal_f64(mu, v, l, tau, 1e-12, 0.6, t, dt, 0)
    s2, _ = oracle.temporal_f64(mu, v, l, tau, 1e-12, 0.6, t)
    np.testing.assert_allclose((small - s2) / dt, v, rtol=1e-9)
    raw, _ = oracle.temporal_f64(mu, v, l, tau, 0.4, 0.6, t, dt, 1)
    np.testing.assert_allclose((raw - base) / dt, v, rtol=1e-12)


def test_opacity_weighted_velocity_integral():
    """Eq. (11): the Gaussian-weighted mean of d mu~/dt, computed by quadrature
    over the oracle's mu~(t), equals v exp(-2 pi^2 rho^2) (the exact value of
    the integral; Eq. (10) is the paper's proxy for it).  Pins the 2 pi / l
    inside the sine and the l / 2 pi amplitude together."""
    import oracle
    mu, v, l, tau, beta = np.zeros(3), np.array([0.3, -0.1, 0.2]), 0.9, 0.2, 0.12
    ts = tau + np.linspace(-10 * beta, 10 * beta, 8001)
    h = 1e-6
    acc = np.zeros(3)
    wsum = 0.0
    for t in ts:
        p, _ = oracle.temporal_f64(mu, v, l, tau, beta, 1.0, t + h)
        m, _ = oracle.temporal_f64(mu, v, l, tau, beta, 1.0, t - h)
        w = math.exp(-0.5 * ((t - tau) / beta) ** 2)
        acc += w * (p - m) / (2 * h)
        wsum += w
    rho = beta / l
    np.testing.assert_allclose(acc / wsum, v * math.exp(-2 * math.pi ** 2 * rho ** 2), rtol=1e-6)


def test_static_special_case_is_time_invariant(orc):
    """Sec. 3.2: v = 0 and rho = +inf reduce PVG to 3DGS: the image no longer
    depends on t."""
    cfg = gen.make_config(0)
    sc = dict(cfg["scene"])
    sc["vel"] = np.zeros_like(sc["vel"])
    sc["beta"] = np.full_like(sc["beta"], 1e8)
    cam = cfg["cameras"][0]
    a = orc.render(sc, cam, 0.1)
    b = orc.render(sc, cam, 0.93)
    assert np.array_equal(a["img"], b["img"]) and np.array_equal(a["n_contrib"], b["n_contrib"])


def test_second_render_reductions(orc):
    """Eq. (12): dt = 0 is the plain render; rho = 1e6 makes v_bar vanish so
    the translated render equals the plain one bitwise."""
    cfg = gen.make_config(0)
    sc, cam = cfg["scene"], cfg["cameras"][0]
    a = orc.render(sc, cam, cfg["t"])
    b = orc.render(sc, cam, cfg["t"], dt=0.0, mode=0)
    assert np.array_equal(a["img"], b["img"])
    s2 = dict(sc)
    s2["beta"] = (s2["period"].astype(np.float64) * 1e6).astype(np.float32)
    c = orc.render(s2, cam, cfg["t"])
    d = orc.render(s2, cam, cfg["t"], dt=0.05, mode=0)
    assert np.array_equal(c["img"], d["img"])
    e = orc.render(sc, cam, cfg["t"], dt=0.05, mode=0)
    assert not np.array_equal(a["img"], e["img"])


# ---------------------------------------------------------------- P4 SH basis
def _real_sh_scipy(l, m, d):
    theta = math.acos(max(-1.0, min(1.0, d[2])))
    phi = math.atan2(d[1], d[0]) % (2 * math.pi)
    if m == 0:
        return sps.sph_harm_y(l, 0, theta, phi).real
    y = sps.sph_harm_y(l, abs(m), theta, phi)
    # scipy includes the Condon-Shortley phase (-1)^m; the basis here does not
    sgn = (-1) ** abs(m)
    return math.sqrt(2.0) * sgn * (y.real if m > 0 else y.imag)


def test_sh_basis_matches_library_real_harmonics():
    """Colour c of Sec. 3.1 as real spherical harmonics, degree <= 3, index
    k = l^2 + l + m, without the Condon-Shortley phase (Y_1 ~ (y, z, x))."""
    import oracle
    rng = np.random.default_rng(5)
    for _ in range(20):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        Y, _ = oracle.sh_basis_f64(d, 3)
        for l in range(4):
            for m in range(-l, l + 1):
                assert Y[l * l + l + m] == pytest.approx(_real_sh_scipy(l, m, d), abs=1e-12)
    Y, _ = oracle.sh_basis_f64(np.array([1.0, 0.0, 0.0]), 3)
    assert Y[0] == pytest.approx(Y00, rel=1e-15)
    assert Y[3] == pytest.approx(math.sqrt(3 / (4 * math.pi)), rel=1e-15)


def test_sh_gram_matrix_is_identity():
    """Orthonormality of the 16 basis functions on the sphere (Gauss-Legendre
    in cos(theta) x uniform in phi)."""
    import oracle
    xg, wg = np.polynomial.legendre.leggauss(24)
    nphi = 48
    G = np.zeros((16, 16))
    for z, wz in zip(xg, wg):
        for j in range(nphi):
            ph = 2 * math.pi * j / nphi
            s = math.sqrt(1 - z * z)
            Y, _ = oracle.sh_basis_f64(np.array([s * math.cos(ph), s * math.sin(ph), z]), 3)
            G += wz * (2 * math.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_gradient_tangential_part():
    """dY/d(dir) of the oracle agrees with finite differences along the sphere."""
    import oracle
    rng = np.random.default_rng(6)
    for _ in range(10):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        _, dY = oracle.sh_basis_f64(d, 3)
        tdir = np.cross(d, rng.standard_normal(3))
        tdir /= np.linalg.norm(tdir)
        h = 1e-6
        yp, _ = oracle.sh_basis_f64((d + h * tdir) / np.linalg.norm(d + h * tdir), 3)
        ym, _ = oracle.sh_basis_f64((d - h * tdir) / np.linalg.norm(d - h * tdir), 3)
        np.testing.assert_allclose((yp - ym) / (2 * h), dY @ tdir, atol=1e-8)


# ---------------------------------------------------------------- P5 EWA
def test_ewa_projection_against_numeric_jacobian():
    """Sec. 3.1 Eq. (2): Sigma' = J W Sigma W^T J^T (+0.3 px^2), J the Jacobian
    of the perspective projection, Sigma = R(q) S S^T R(q)^T (unit quaternion
    q, scale s).  J W is taken by central differences of the projected mean
    and R(q) from scipy's quaternion conversion."""
    import oracle
    rng = np.random.default_rng(8)
    for k in range(6):
        cam = gen.yaw_camera(128, 96, float(rng.uniform(-40, 40)), (0.3, -0.2, -1.0))
        mu = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(3, 8)])
        s = rng.uniform(0.05, 0.4, 3)
        q = rng.standard_normal(4) * (1.0 + k)  # any nonzero norm
        m, J, cov = oracle.project_f64(mu, s, q, cam)
        h = 1e-6
        JW = np.zeros((2, 3))
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            mp, _, _ = oracle.project_f64(mu + e, s, q, cam)
            mm, _, _ = oracle.project_f64(mu - e, s, q, cam)
            JW[:, c] = (mp - mm) / (2 * h)
        qn = q / np.linalg.norm(q)
        Rq = Rotation.from_quat([qn[1], qn[2], qn[3], qn[0]]).as_matrix()  # scipy: (x, y, z, w)
        Sig = Rq @ np.diag(s ** 2) @ Rq.T
        expect = JW @ Sig @ JW.T + 0.3 * np.eye(2)
        np.testing.assert_allclose([cov[0], cov[1], cov[2]], [expect[0, 0], expect[0, 1], expect[1, 1]],
                                   rtol=2e-6, atol=1e-7)


# ---------------------------------------------------------------- P6, P7 structure
@pytest.mark.parametrize("seed", [0, 11, 12])
def test_bruteforce_equals_tiled(orc, seed):
    """Tiling, instance emission and the global sort only build each pixel's
    depth-ordered list (Sec. 3.1): a per-pixel brute force without tiles gives
    the same image bit for bit."""
    sc = gen.make_scene(600, seed, sh_degree=1)
    cam = gen.make_camera(80, 56)  # ragged: 5 x 3.5 tiles
    r = orc.render(sc, cam, 0.37, dt=0.05, bg=(0.1, 0.0, 0.3))
    img, T, nc = orc.render_bruteforce_f32(r["pre"], cam, 0.37, 0.05, 0, (0.1, 0.0, 0.3))
    assert np.array_equal(img, r["img"]) and np.array_equal(T, r["final_T"]) and np.array_equal(nc, r["n_contrib"])


def test_instances_sorted_by_tile_depth_index(orc):
    """Ordering by camera-space depth (Sec. 3.1) per 16x16 tile, ties by index:
    the oracle's sorted instances equal numpy's lexsort of (tile, depth bits,
    index) built from the tile rectangles; the count is the sum of their areas."""
    cfg = gen.make_config(0)
    cam = cfg["cameras"][0]
    pre = orc.preprocess_f32(cfg["scene"], cam, cfg["t"])
    # force depth ties
    pre["depth"][::7] = pre["depth"][3]
    bins = orc.bin_sort(pre, cam)
    GX = 8
    tiles, dbits, idx = [], [], []
    for i in np.nonzero(pre["radius"] > 0)[0]:
        x0, y0, x1, y1 = pre["rect"][i]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                tiles.append(ty * GX + tx)
                dbits.append(pre["depth"][i].view(np.uint32))
                idx.append(i)
    tiles, dbits, idx = map(np.array, (tiles, dbits, idx))
    order = np.lexsort((idx, dbits, tiles))
    assert bins["M"] == int(((pre["rect"][:, 2] - pre["rect"][:, 0]) * (pre["rect"][:, 3] - pre["rect"][:, 1]))
                             [pre["radius"] > 0].sum())
    assert np.array_equal(bins["inst_gauss"], idx[order])
    assert np.array_equal(bins["inst_tile"], tiles[order])
    counts = np.bincount(tiles, minlength=48)
    assert np.array_equal(bins["ranges"][:, 1] - bins["ranges"][:, 0], counts)


# ---------------------------------------------------------------- P8 gradients
def _fd_check(orc, sc, cam, t, dt, mode, bg, fields=None, sample=None, seed=0, tol=1e-6, channels=False):
    pre = orc.preprocess_f32(sc, cam, t, dt, mode, bg)
    bins = orc.bin_sort(pre, cam)
    s64 = orc.scene64(sc)
    W, H = cam["width"], cam["height"]
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((3, H, W))
    wD = rng.standard_normal((H, W)) * 0.1 if channels else None  # depths are O(10): keep the terms comparable
    wT = rng.standard_normal((H, W)) if channels else None
    wF = rng.standard_normal((4, H, W)) if channels else None
    grads, _ = orc.backward_f64(s64, cam, t, dt, mode, bg, pre, bins, w, dD=wD, dT=wT, dF=wF)
    GX, GY = orc.grid(cam)
    vis = np.nonzero(pre["radius"] > 0)[0]
    assert vis.size > 0
    checked = 0
    for f in (fields or orc.FIELDS):
        arr = s64[f].reshape(-1, sc["n"])
        g = grads[f].reshape(-1, sc["n"])
        rms = np.sqrt(np.mean(g[:, vis] ** 2))
        entries = [(r, i) for r in range(arr.shape[0]) for i in vis]
        if sample is not None and len(entries) > sample:
            entries = [entries[j] for j in rng.choice(len(entries), sample, replace=False)]
        for r, i in entries:
            x0, y0, x1, y1 = pre["rect"][i]
            tm = np.zeros((GY, GX), np.uint8)
            tm[y0:y1, x0:x1] = 1
            old = arr[r, i]
            h = 1e-4 * max(1.0, abs(old))
            L = {}
            for k in (-2, -1, 1, 2):
                arr[r, i] = old + k * h
                L[k] = orc.render_f64(s64, cam, t, dt, mode, bg, pre, bins, tile_mask=tm.reshape(-1), w=w,
                                      want_img=False, wD=wD, wT=wT, wF=wF)[0]
            arr[r, i] = old
            fd = (8 * (L[1] - L[-1]) - (L[2] - L[-2])) / (12 * h)
            err = abs(fd - g[r, i]) / max(abs(g[r, i]), 1e-2 * rms)
            assert err <= tol, (f, r, i, fd, g[r, i], rms)
            checked += 1
    return checked


@pytest.mark.parametrize("dt,mode", [(0.0, 0), (0.05, 0), (0.05, 1)])
def test_adjoint_matches_finite_differences_tiny(orc, dt, mode):
    """Finite differences of the FP64 image on a fixed discrete structure
    against the FP64 adjoint, for every parameter of every visible Gaussian
    (Sec. 3.2 parameter set {mu, q, s, o, c, tau, beta, v} and l), for the
    plain render and for the flow-translated render of Eq. (12)."""
    sc = gen.make_scene(30, 7, sh_degree=3)
    cam = gen.yaw_camera(64, 48, 10.0, (0.2, 0.1, -0.5))
    n = _fd_check(orc, sc, cam, 0.45, dt, mode, (0.1, 0.2, 0.3))
    assert n > 500


@pytest.mark.parametrize("dt,mode", [(0.0, 0), (0.05, 0)])
def test_channel_adjoint_matches_finite_differences_tiny(orc, dt, mode):
    """Flexible rendering (Sec. 3.1): the blended depth channel sum T alpha z,
    the velocity map sum T alpha v~ with v~ = v exp(-beta / (2 l)) and the
    staticness map sum T alpha beta / l, and the final transmittance (the
    rendered opacity O is 1 - final_T) enter the loss with their own upstream
    gradients; finite differences of that loss against the FP64 adjoint for
    every parameter of every visible Gaussian."""
    sc = gen.make_scene(30, 7, sh_degree=3)
    cam = gen.yaw_camera(64, 48, 10.0, (0.2, 0.1, -0.5))
    n = _fd_check(orc, sc, cam, 0.45, dt, mode, (0.1, 0.2, 0.3), channels=True)
    assert n > 500


def test_depth_channel_closed_form(orc):
    """With every Gaussian at one camera depth z0 the blended depth is
    z0 * sum T alpha = z0 * (1 - final_T) at every pixel (FP64 to rounding,
    the FP32 image path to a few ulps), and a pixel no Gaussian reaches has
    depth 0 and final_T 1."""
    cfg = gen.make_config(0)
    sc = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in cfg["scene"].items()}
    cam = cfg["cameras"][0]
    assert np.allclose(np.asarray(cam["R"], np.float64).reshape(3, 3), np.eye(3)) and not np.any(cam["T"])
    z0 = 6.5
    sc["mu"][2] = z0
    sc["vel"][2] = 0.0  # the vibration leaves z unchanged
    pre = orc.preprocess_f32(sc, cam, cfg["t"])
    assert np.all(pre["depth"][pre["radius"] > 0] == np.float32(z0))
    bins = orc.bin_sort(pre, cam)
    img, T, nc, D = orc.render_f32(pre, bins, cam, cfg["t"], want_depth=True)
    np.testing.assert_allclose(D, z0 * (1.0 - T.astype(np.float64)), rtol=1e-5, atol=1e-5)
    empty = nc == 0
    assert np.all(D[empty] == 0.0) and np.all(T[empty] == 1.0)
    _, _, T64, D64 = orc.render_f64(orc.scene64(sc), cam, cfg["t"], 0.0, 0, (0, 0, 0), pre, bins, want_depth=True)
    np.testing.assert_allclose(D64, z0 * (1.0 - T64), rtol=1e-12, atol=1e-12)


def test_normalized_depth_closed_form_and_bounds(orc):
    """Normalized depth (Sec. 3.1): with every Gaussian at one camera depth z0
    it is z0 on every pixel a Gaussian reaches and 0 elsewhere; on a random
    scene it is a convex combination of the contributors' depths, so it lies
    between the smallest and the largest visible depth."""
    cfg = gen.make_config(0)
    cam, t = cfg["cameras"][0], cfg["t"]
    sc = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in cfg["scene"].items()}
    z0 = 6.5
    sc["mu"][2] = z0
    sc["vel"][2] = 0.0
    sc = gen.subset_scene(sc, np.arange(40))  # leaves part of the image empty
    pre = orc.preprocess_f32(sc, cam, t)
    bins = orc.bin_sort(pre, cam)
    _, _, T64, D64 = orc.render_f64(orc.scene64(sc), cam, t, 0.0, 0, (0, 0, 0), pre, bins, want_depth=True)
    Dn = orc.normalized_depth_f64(D64, T64)
    _, _, nc = orc.render_f32(pre, bins, cam, t)
    hit = nc > 0
    assert 0.05 < hit.mean() < 0.95
    np.testing.assert_allclose(Dn[hit], z0, rtol=1e-12)
    assert np.all(Dn[~hit] == 0.0)
    # a random scene: sum T alpha z / sum T alpha within [min z, max z]
    sc = cfg["scene"]
    pre = orc.preprocess_f32(sc, cam, t)
    bins = orc.bin_sort(pre, cam)
    _, _, T64, D64 = orc.render_f64(orc.scene64(sc), cam, t, 0.0, 0, (0, 0, 0), pre, bins, want_depth=True)
    Dn = orc.normalized_depth_f64(D64, T64)
    _, _, nc = orc.render_f32(pre, bins, cam, t)
    vis = pre["radius"] > 0
    zmin, zmax = float(pre["depth"][vis].min()), float(pre["depth"][vis].max())
    hit = nc > 0
    assert np.all(Dn[hit] >= zmin * (1 - 1e-6)) and np.all(Dn[hit] <= zmax * (1 + 1e-6))
    assert Dn[hit].std() > 0.1  # not a constant


def test_normalized_depth_adjoint_matches_finite_differences(orc):
    """L = sum w img + sum g D / A (A = sum T alpha): finite differences of the
    FP64 render against the FP64 adjoint fed with normalized_depth_bwd_f64's
    (dD, dT), sampled entries of every field of the visible Gaussians."""
    sc = gen.make_scene(30, 7, sh_degree=1)
    cam = gen.yaw_camera(64, 48, 10.0, (0.2, 0.1, -0.5))
    t = 0.45
    pre = orc.preprocess_f32(sc, cam, t)
    bins = orc.bin_sort(pre, cam)
    s64 = orc.scene64(sc)
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(4)
    w = rng.standard_normal((3, H, W))
    g = rng.standard_normal((H, W))

    def loss():
        _, img, T, D = orc.render_f64(s64, cam, t, 0.0, 0, (0, 0, 0), pre, bins, want_depth=True)
        return float(np.sum(w * img) + np.sum(g * orc.normalized_depth_f64(D, T)))

    _, _, T0, D0 = orc.render_f64(s64, cam, t, 0.0, 0, (0, 0, 0), pre, bins, want_depth=True)
    dD, dT = orc.normalized_depth_bwd_f64(g, D0, T0)
    grads, _ = orc.backward_f64(s64, cam, t, 0.0, 0, (0, 0, 0), pre, bins, w, dD=dD, dT=dT)
    vis = np.nonzero(pre["radius"] > 0)[0]
    checked = 0
    for f in orc.FIELDS:
        arr = s64[f].reshape(-1, sc["n"])
        gr = grads[f].reshape(-1, sc["n"])
        rms = np.sqrt(np.mean(gr[:, vis] ** 2))
        entries = [(r, i) for r in range(arr.shape[0]) for i in vis]
        for j in rng.choice(len(entries), min(25, len(entries)), replace=False):
            r, i = entries[j]
            old = arr[r, i]
            h = 1e-4 * max(1.0, abs(old))
            L = {}
            for k in (-2, -1, 1, 2):
                arr[r, i] = old + k * h
                L[k] = loss()
            arr[r, i] = old
            fd = (8 * (L[1] - L[-1]) - (L[2] - L[-2])) / (12 * h)
            assert abs(fd - gr[r, i]) <= 1e-6 * max(abs(gr[r, i]), 1e-2 * rms), (f, r, i, fd, gr[r, i])
            checked += 1
    assert checked >= 150


def test_velocity_and_staticness_maps_closed_form(orc):
    """With v = 0 the velocity map is exactly 0; with beta / l = rho0 for
    every Gaussian the staticness map is rho0 * (1 - final_T) (FP64 to
    rounding, FP32 to a few ulps); and the velocity map of one Gaussian alone
    over a pixel is its T alpha v exp(-beta / (2 l))."""
    cfg = gen.make_config(0)
    cam, t = cfg["cameras"][0], cfg["t"]
    sc = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in cfg["scene"].items()}
    sc["vel"][:] = 0.0
    rho0 = 0.625
    sc["beta"][:] = np.float32(rho0) * sc["period"]
    pre = orc.preprocess_f32(sc, cam, t)
    vis = pre["radius"] > 0
    assert np.all(pre["feat"][vis, :3] == 0.0)
    bins = orc.bin_sort(pre, cam)
    img, T, nc, F = orc.render_f32(pre, bins, cam, t, want_feat=True)
    assert np.all(F[:3] == 0.0)
    np.testing.assert_allclose(F[3], pre["feat"][vis, 3].max() * (1.0 - T.astype(np.float64)), rtol=1e-5,
                               atol=1e-5)
    assert np.allclose(pre["feat"][vis, 3], rho0, rtol=1e-6)
    # one Gaussian: the map at its centre pixel is alpha v~ (T = 1 in front of it)
    full = orc.preprocess_f32(cfg["scene"], cam, t)
    inside = np.nonzero((full["radius"] > 0) & (full["xy"][:, 0] > 4) & (full["xy"][:, 0] < cam["width"] - 4)
                        & (full["xy"][:, 1] > 4) & (full["xy"][:, 1] < cam["height"] - 4)
                        & (full["conic_op"][:, 3] > 0.1))[0]
    one = gen.subset_scene(cfg["scene"], inside[:1])
    p1 = orc.preprocess_f32(one, cam, t)
    b1 = orc.bin_sort(p1, cam)
    _, T1, n1, F1 = orc.render_f32(p1, b1, cam, t, want_feat=True)
    x, y = int(round(float(p1["xy"][0, 0]))), int(round(float(p1["xy"][0, 1])))
    assert n1[y, x] == 1
    a = 1.0 - float(T1[y, x])
    e = np.exp(-0.5 * float(one["beta"][0]) / float(one["period"][0]))
    np.testing.assert_allclose(F1[:3, y, x], a * e * one["vel"][:, 0].astype(np.float64), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(F1[3, y, x], a * float(one["beta"][0]) / float(one["period"][0]), rtol=1e-5)


def test_channel_adjoint_linear(orc):
    """The adjoint of image, depth and final_T gradients together is the sum
    of the three adjoints taken one at a time."""
    cfg = gen.make_config(0)
    cam = cfg["cameras"][0]
    sc, t = cfg["scene"], cfg["t"]
    pre = orc.preprocess_f32(sc, cam, t, 0.05)
    bins = orc.bin_sort(pre, cam)
    s64 = orc.scene64(sc)
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(5)
    w, wD, wT = rng.standard_normal((3, H, W)), rng.standard_normal((H, W)), rng.standard_normal((H, W))
    zero = np.zeros((3, H, W))
    g_all, g2_all = orc.backward_f64(s64, cam, t, 0.05, 0, (0, 0, 0), pre, bins, w, dD=wD, dT=wT)
    parts = [orc.backward_f64(s64, cam, t, 0.05, 0, (0, 0, 0), pre, bins, w),
             orc.backward_f64(s64, cam, t, 0.05, 0, (0, 0, 0), pre, bins, zero, dD=wD),
             orc.backward_f64(s64, cam, t, 0.05, 0, (0, 0, 0), pre, bins, zero, dT=wT)]
    for f in orc.FIELDS:
        tot = sum(p[0][f] for p in parts)
        np.testing.assert_allclose(g_all[f], tot, rtol=1e-9, atol=1e-12 * (1 + np.abs(tot).max()))
    assert np.any(parts[1][1][:, 9] != 0) and not np.any(parts[2][1][:, 9])  # only the depth term reaches d z


def test_adjoint_matches_finite_differences_config1_subset(orc):
    """The 960x640, degree-3 differentiation workload on a 500-Gaussian subset
    of its scene (Gaussians that touch tiles), sampled entries of every field."""
    cfg = gen.make_config(1, n=20_000)
    cam = cfg["cameras"][0]
    pre = orc.preprocess_f32(cfg["scene"], cam, cfg["t"])
    rng = np.random.default_rng(2)
    idx = np.sort(rng.choice(np.nonzero(pre["tiles"] > 0)[0], 500, replace=False))
    sub = gen.subset_scene(cfg["scene"], idx)
    n = _fd_check(orc, sub, cam, cfg["t"], 0.05, 0, (0.0, 0.0, 0.0), sample=12, seed=3)
    assert n >= 9 * 12


def test_adjoint_linear_in_upstream_gradient(orc):
    """The adjoint is linear in dL/dimage: grad(a w1 + b w2) = a grad(w1) + b grad(w2)."""
    sc = gen.make_scene(40, 9, sh_degree=2)
    cam = gen.make_camera(48, 32)
    pre = orc.preprocess_f32(sc, cam, 0.5, 0.05, 0, (0, 0, 0))
    bins = orc.bin_sort(pre, cam)
    s64 = orc.scene64(sc)
    rng = np.random.default_rng(1)
    w1, w2 = rng.standard_normal((2, 3, 32, 48))
    g1, _ = orc.backward_f64(s64, cam, 0.5, 0.05, 0, (0, 0, 0), pre, bins, w1)
    g2, _ = orc.backward_f64(s64, cam, 0.5, 0.05, 0, (0, 0, 0), pre, bins, w2)
    g3, _ = orc.backward_f64(s64, cam, 0.5, 0.05, 0, (0, 0, 0), pre, bins, 2 * w1 - 3 * w2)
    for f in orc.FIELDS:
        np.testing.assert_allclose(g3[f], 2 * g1[f] - 3 * g2[f], atol=1e-12 * (1 + np.abs(g3[f]).max()))


def test_fp64_image_close_to_fp32(orc):
    """The FP64 evaluation on the FP32 structure is the same image up to FP32 rounding."""
    cfg = gen.make_config(0)
    cam = cfg["cameras"][0]
    r = orc.render(cfg["scene"], cam, cfg["t"])
    _, img64, T64 = orc.render_f64(orc.scene64(cfg["scene"]), cam, cfg["t"], 0.0, 0, (0, 0, 0), r["pre"],
                                   r["bins"])
    assert np.abs(img64 - r["img"]).max() < 2e-6
    assert np.abs(T64 - r["final_T"]).max() < 2e-6


def test_tile_masked_adjoint_equals_full(orc):
    """The adjoint restricted to a tile mask equals the full adjoint when the
    image gradient vanishes outside the mask (the mask only skips work)."""
    import gen
    scene = gen.make_scene(300, 17, sh_degree=2)
    cam = gen.make_camera(96, 64)
    t = 0.4
    pre = orc.preprocess_f32(scene, cam, t)
    bins = orc.bin_sort(pre, cam)
    GX, GY = orc.grid(cam)
    mask = np.zeros(GX * GY, np.uint8)
    mask[[3, 9, 14]] = 1
    keep = np.repeat(np.repeat(mask.reshape(GY, GX), 16, 0), 16, 1)[:64, :96].astype(bool)
    dimg = np.random.default_rng(3).standard_normal((3, 64, 96)) * keep
    sc64 = orc.scene64(scene)
    full, g_full = orc.backward_f64(sc64, cam, t, 0.0, 0, (0, 0, 0), pre, bins, dimg)
    part, g_part = orc.backward_f64(sc64, cam, t, 0.0, 0, (0, 0, 0), pre, bins, dimg, tile_mask=mask)
    assert np.array_equal(g_full, g_part)
    for f in full:
        assert np.array_equal(full[f], part[f]), f
    assert np.abs(g_full).max() > 0


def test_feature_in_place_of_colour_closed_form(orc):
    """Semantic rendering (Sec. 4.1) composites per-Gaussian vectors like the
    colour: a constant vector f gives f (1 - final_T) at every pixel."""
    cfg = gen.make_config(0)
    sc, cam, t = cfg["scene"], cfg["cameras"][0], cfg["t"]
    pre = orc.preprocess_f32(sc, cam, t)
    bins = orc.bin_sort(pre, cam)
    f = np.array([0.2, -0.5, 0.9])
    col = np.tile(f, (sc["n"], 1))
    _, img, T = orc.render_f64(orc.scene64(sc), cam, t, 0.0, 0, (0, 0, 0), pre, bins, colour=col)
    np.testing.assert_allclose(img, f[:, None, None] * (1.0 - T)[None], rtol=1e-12, atol=1e-14)


def test_feature_in_place_of_colour_adjoint_fd(orc):
    """With per-Gaussian values in place of the colour (any sign): finite
    differences of sum w img against the adjoint, with respect to those
    values (g2d[:, 6:9]) and to the geometry; nothing reaches the SH."""
    sc = gen.make_scene(30, 7, sh_degree=2)
    cam = gen.yaw_camera(64, 48, 10.0, (0.2, 0.1, -0.5))
    t = 0.45
    pre = orc.preprocess_f32(sc, cam, t)
    bins = orc.bin_sort(pre, cam)
    s64 = orc.scene64(sc)
    rng = np.random.default_rng(8)
    col = rng.standard_normal((sc["n"], 3))
    w = rng.standard_normal((3, cam["height"], cam["width"]))
    grads, g2d = orc.backward_f64(s64, cam, t, 0.0, 0, (0, 0, 0), pre, bins, w, colour=col)
    assert not np.any(grads["sh"])

    def loss(c=col):
        return orc.render_f64(s64, cam, t, 0.0, 0, (0, 0, 0), pre, bins, w=w, want_img=False, colour=c)[0]

    vis = np.nonzero(pre["radius"] > 0)[0]
    for i in vis[:8]:
        for ch in range(3):
            cp, cm = col.copy(), col.copy()
            cp[i, ch] += 1e-6
            cm[i, ch] -= 1e-6
            fd = (loss(cp) - loss(cm)) / 2e-6
            assert abs(fd - g2d[i, 6 + ch]) <= 1e-7 * max(1.0, abs(fd)), (i, ch, fd, g2d[i, 6 + ch])
    rms = {f: np.sqrt(np.mean(grads[f].reshape(-1, sc["n"])[:, vis] ** 2)) for f in ("mu", "opacity", "scale")}
    for f in ("mu", "opacity", "scale"):
        arr = s64[f].reshape(-1, sc["n"])
        g = grads[f].reshape(-1, sc["n"])
        for i in vis[:6]:
            old = arr[0, i]
            h = 1e-5 * max(1.0, abs(old))
            arr[0, i] = old + h
            lp = loss()
            arr[0, i] = old - h
            lm = loss()
            arr[0, i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[0, i]) <= 1e-5 * max(abs(g[0, i]), 1e-2 * rms[f]), (f, i, fd, g[0, i])
