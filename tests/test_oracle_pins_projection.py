"""Pins of the oracle's projection branches that the on-axis closed forms do
not reach (Sec. 3.1, Eq. (2): the EWA projection of the 3D covariance; Eq. (3):
alpha of the projected 2D Gaussian):

- the Jacobian guard: a mean seen beyond 1.3x the half field of view gets the
  Jacobian of the pinhole map at the point clamped to that band, while its 2D
  mean stays the true projection;
- the screen radius of an anisotropic splat, ceil(3 sqrt(lambda_max)), where
  the eigenvalue discriminant is above its 0.1 floor;
- the image of one rotated anisotropic splat, which depends on the inversion
  of the 2D covariance and on the sign of its cross term.

Every expected value comes from numpy / scipy in FP64, never from the oracle:
the Jacobian by central differences of the pinhole map, R(q) from scipy's
quaternion conversion, the largest eigenvalue from numpy.linalg.eigvalsh and
the 2D Gaussian evaluated pixel by pixel.

The last test plants, in copies of the oracle's source, each mistake these pins
exist to catch (the guard without its half, the radius without the square root
of the discriminant, the sign of the conic's cross term in either of its two
places, the conic's diagonal swapped), and five more that the main pin module
must catch (the sine's amplitude, a sign in the EWA product, one rotation
entry, the signs of dL/dB and dL/dl), and checks that the pin then fails."""
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import gen

TILE = 16
GUARD = 1.3
DILATION = 0.3
Y00 = 0.5 / math.sqrt(math.pi)


# ------------------------------------------------------------ FP64 references
def _cam_rt(cam):
    return np.asarray(cam["R"], np.float64).reshape(3, 3), np.asarray(cam["T"], np.float64)


def pinhole(cam, p):
    """Pixel-space projection of a camera-frame point, in the sampling frame
    (pixel (i, j) is sampled where the projection minus (0.5, 0.5) is (i, j))."""
    return np.array([cam["fx"] * p[0] / p[2] + cam["cx"] - 0.5, cam["fy"] * p[1] / p[2] + cam["cy"] - 0.5])


def guard_point(cam, p):
    """p with its x/z and y/z clamped to 1.3x the half field of view."""
    limx = GUARD * 0.5 * cam["width"] / cam["fx"]
    limy = GUARD * 0.5 * cam["height"] / cam["fy"]
    return np.array([np.clip(p[0] / p[2], -limx, limx) * p[2], np.clip(p[1] / p[2], -limy, limy) * p[2], p[2]])


def jacobian_fd(cam, p):
    """d pinhole / d p by central differences."""
    J = np.zeros((2, 3))
    for c in range(3):
        h = 1e-6 * max(1.0, abs(p[c]))
        e = np.zeros(3)
        e[c] = h
        J[:, c] = (pinhole(cam, p + e) - pinhole(cam, p - e)) / (2.0 * h)
    return J


def sigma3d(s, q):
    qn = np.asarray(q, np.float64) / np.linalg.norm(q)
    Rq = Rotation.from_quat([qn[1], qn[2], qn[3], qn[0]]).as_matrix()  # scipy order (x, y, z, w)
    return Rq @ np.diag(np.asarray(s, np.float64) ** 2) @ Rq.T


def ewa(cam, mu, s, q, guard=True):
    """(2D mean, dilated 2D covariance) of Eq. (2): J (at the guard-clamped
    point) W Sigma W^T J^T + 0.3 I, the mean at the unclamped point."""
    R, T = _cam_rt(cam)
    p = R @ np.asarray(mu, np.float64) + T
    J = jacobian_fd(cam, guard_point(cam, p) if guard else p)
    JW = J @ R
    return pinhole(cam, p), JW @ sigma3d(s, q) @ JW.T + DILATION * np.eye(2)


def conic_of(cov):
    Q = np.linalg.inv(cov)
    return np.array([Q[0, 0], Q[0, 1], Q[1, 1]])


def world_mean(cam, p):
    R, T = _cam_rt(cam)
    return R.T @ (np.asarray(p, np.float64) - T)


def one_gaussian(mu, s, q, o=0.8, sh0=(0.9, -0.3, 0.2)):
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    return {"n": 1, "sh_degree": 0, "mu": f(np.reshape(mu, (3, 1))), "scale": f(np.reshape(s, (3, 1))),
            "rot": f(np.reshape(q, (4, 1))), "sh": f(np.reshape(sh0, (1, 3, 1))), "opacity": f([o]),
            "vel": f(np.zeros((3, 1))), "period": f([1.0]), "tau": f([0.5]), "beta": f([1e8])}


def f32_scene_values(sc):
    """The parameters as the oracle sees them (rounded to FP32)."""
    return (sc["mu"][:, 0].astype(np.float64), sc["scale"][:, 0].astype(np.float64),
            sc["rot"][:, 0].astype(np.float64))


# ------------------------------------------------------------ the pins
# (camera-frame direction x/z, y/z, depth z, scale, quaternion seed): each
# mean lies beyond the guard band on the named side(s), each splat large
# enough that its rectangle still reaches the image
GUARD_CASES = {
    "x beyond +": ((1.25, 0.10), 6.0, (2.5, 0.6, 0.4), 1),
    "x and y beyond -": ((-1.40, -0.90), 5.0, (3.0, 2.0, 1.0), 2),
    "y beyond +": ((0.30, 1.00), 6.0, (2.0, 2.2, 0.5), 3),
}


def pin_guard(orc, name):
    (ux, uy), z, s, seed = GUARD_CASES[name]
    cam = gen.yaw_camera(256, 192, 10.0, (0.5, -0.2, -1.0))
    q = np.random.default_rng(seed).standard_normal(4)
    sc = one_gaussian(world_mean(cam, [ux * z, uy * z, z]), s, q)
    mu, s32, q32 = f32_scene_values(sc)
    pre = orc.preprocess_f32(sc, cam, 0.5)
    assert pre["radius"][0] > 0, "the case must stay visible"
    m, cov = ewa(cam, mu, s32, q32, guard=True)
    _, cov_free = ewa(cam, mu, s32, q32, guard=False)
    want, free = conic_of(cov), conic_of(cov_free)
    scale = np.abs(want).max()
    # the case exercises the guard: the unguarded Jacobian gives another conic
    assert np.abs(free - want).max() > 5e-2 * scale, name
    got = pre["conic_op"][0, :3].astype(np.float64)
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-5 * scale, err_msg=name)
    # the 2D mean is the true projection, not the clamped point's
    np.testing.assert_allclose(pre["xy"][0].astype(np.float64), m, rtol=2e-6, atol=2e-4, err_msg=name)


@pytest.mark.parametrize("name", list(GUARD_CASES))
def test_jacobian_guard_band(orc, name):
    """Sec. 3.1 Eq. (2) with the guard band: J is the Jacobian of the pinhole
    map at the mean clamped to 1.3x the half field of view (x/z and y/z each);
    the splat's centre stays at the true projection."""
    pin_guard(orc, name)


def _radius_cases():
    rng = np.random.default_rng(21)
    cam = gen.yaw_camera(640, 480, -20.0, (1.0, 0.5, -2.0))
    cases = []
    for _ in range(60):
        z = rng.uniform(3.0, 12.0)
        p = [rng.uniform(-0.45, 0.45) * z, rng.uniform(-0.35, 0.35) * z, z]
        a = math.exp(rng.normal(-1.0, 0.4))
        s = np.array([a, a / rng.uniform(3.0, 8.0), a / rng.uniform(3.0, 8.0)])
        cases.append((world_mean(cam, p), s, rng.standard_normal(4)))
    return cam, cases


def pin_radius(orc):
    cam, cases = _radius_cases()
    GX, GY = (cam["width"] + TILE - 1) // TILE, (cam["height"] + TILE - 1) // TILE
    checked = 0
    for mu0, s0, q0 in cases:
        sc = one_gaussian(mu0, s0, q0)
        mu, s, q = f32_scene_values(sc)
        m, cov = ewa(cam, mu, s, q)
        a, b, c = cov[0, 0], cov[0, 1], cov[1, 1]
        if ((a + c) / 2) ** 2 - (a * c - b * b) < 0.2:  # the 0.1 floor would act: not this pin's case
            continue
        x = 3.0 * math.sqrt(np.linalg.eigvalsh(cov)[-1])
        if abs(x - round(x)) < 1e-4 * x:
            continue
        r = math.ceil(x)
        pre = orc.preprocess_f32(sc, cam, 0.5)
        assert pre["radius"][0] == r, (pre["radius"][0], r, x)
        edges = [(m[0] - r) / TILE, (m[1] - r) / TILE, (m[0] + r + TILE - 1) / TILE, (m[1] + r + TILE - 1) / TILE]
        if min(abs(e - round(e)) for e in edges) < 1e-4:
            continue
        rect = [min(max(math.floor(e), 0), hi) for e, hi in zip(edges, (GX, GY, GX, GY))]
        assert list(pre["rect"][0]) == rect, (list(pre["rect"][0]), rect)
        assert pre["tiles"][0] == (rect[2] - rect[0]) * (rect[3] - rect[1])
        checked += 1
    assert checked >= 30, checked


def test_anisotropic_radius_from_largest_eigenvalue(orc):
    """The screen radius of an anisotropic splat is ceil(3 sqrt(lambda_max))
    of its dilated 2D covariance (numpy's eigenvalues) wherever the
    discriminant exceeds the 0.1 floor, and its tile rectangle and tile count
    follow from that radius and the true 2D mean."""
    pin_radius(orc)


ROTATED = {  # camera-frame mean, scale, quaternion, opacity, degree-0 colour
    "oblique": ((0.4, -0.3, 6.0), (0.55, 0.09, 0.14), (0.8, 0.3, -0.2, 0.45), 0.8, (0.9, -0.3, 0.2)),
    "steep": ((-0.8, 0.5, 4.5), (0.06, 0.45, 0.2), (0.3, -0.6, 0.5, 0.55), 0.95, (0.2, 0.7, -0.5)),
}


def pin_rotated_image(orc, name):
    pc, s0, q0, o, sh0 = ROTATED[name]
    cam = gen.yaw_camera(128, 96, 5.0, (0.2, 0.1, -0.5))
    sc = one_gaussian(world_mean(cam, pc), s0, q0, o, sh0)
    mu, s, q = f32_scene_values(sc)
    m, cov = ewa(cam, mu, s, q)
    assert abs(cov[0, 1]) > 0.2 * math.sqrt(cov[0, 0] * cov[1, 1]), "the case needs a strong cross term"
    Qm = np.linalg.inv(cov)
    W, H = cam["width"], cam["height"]
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    dx, dy = m[0] - xs, m[1] - ys
    power = -0.5 * (Qm[0, 0] * dx * dx + Qm[1, 1] * dy * dy) - Qm[0, 1] * dx * dy
    raw = float(np.float32(o)) * np.exp(power)
    alpha = np.minimum(0.99, raw)
    col = np.maximum(0.0, Y00 * np.asarray(sc["sh"][0, :, 0], np.float64) + 0.5)
    r = math.ceil(3.0 * math.sqrt(np.linalg.eigvalsh(cov)[-1]))
    GX, GY = W // TILE, H // TILE
    x0, y0 = max(0, math.floor((m[0] - r) / TILE)), max(0, math.floor((m[1] - r) / TILE))
    x1, y1 = min(GX, math.floor((m[0] + r + TILE - 1) / TILE)), min(GY, math.floor((m[1] + r + TILE - 1) / TILE))
    tx, ty = xs.astype(int) // TILE, ys.astype(int) // TILE
    listed = (tx >= x0) & (tx < x1) & (ty >= y0) & (ty < y1)
    keep = listed & (alpha >= 1.0 / 255.0)
    expect = np.where(keep[None], alpha[None] * col[:, None, None], 0.0)
    # pixels whose alpha sits at a threshold could take either branch in FP32
    edge = (np.abs(alpha * 255.0 - 1.0) < 1e-3) | (np.abs(raw - 0.99) < 1e-4)
    assert keep.sum() > 200, keep.sum()
    r32 = orc.render(sc, cam, 0.5)
    assert r32["pre"]["radius"][0] == r
    err32 = np.abs(r32["img"].astype(np.float64) - expect)[:, ~edge].max()
    assert err32 <= 1e-5, (name, err32)
    L, img64, _ = orc.render_f64(orc.scene64(sc), cam, 0.5, 0.0, 0, (0, 0, 0), r32["pre"], r32["bins"])
    err64 = np.abs(img64 - expect)[:, ~edge].max()
    assert err64 <= 1e-8, (name, err64)


@pytest.mark.parametrize("name", list(ROTATED))
def test_rotated_anisotropic_splat_image(orc, name):
    """Eq. (3) for one rotated anisotropic splat: every pixel of its listed
    tiles is min(0.99, o exp(-1/2 d^T Sigma'^-1 d)) times its colour where
    that alpha is at least 1/255, and 0 elsewhere, with Sigma' the EWA
    covariance of Eq. (2) (numeric Jacobian, scipy rotation); the FP32 image
    to 1e-5 and the FP64 image to 1e-8."""
    pin_rotated_image(orc, name)


# ------------------------------------------------------------ planted mistakes
def _all_guard(orc):
    for name in GUARD_CASES:
        pin_guard(orc, name)


def _all_rotated(orc):
    for name in ROTATED:
        pin_rotated_image(orc, name)


MUTATIONS = {
    "guard band without the half": (
        [("R(1.3f) * ((R(0.5f) * R(cam.W)) / fx)", "R(1.3f) * (R(cam.W) / fx)"),
         ("R(1.3f) * ((R(0.5f) * R(cam.H)) / fy)", "R(1.3f) * (R(cam.H) / fy)")], _all_guard),
    "radius without the square root": (
        [("mid + std::sqrt(std::max(R(0.1f), mid * mid - it.det))", "mid + std::max(R(0.1f), mid * mid - it.det)")],
        pin_radius),
    "sign of B in the conic": ([("s.B = -cb / it.det;", "s.B = cb / it.det;")], _all_rotated),
    "sign of the cross term in alpha": ([("- d.B * (dx * dy)", "+ d.B * (dx * dy)")], _all_rotated),
    "conic diagonal swapped": ([("s.A = cc / it.det;", "s.A = ca / it.det;"),
                                ("s.C = ca / it.det;", "s.C = cc / it.det;")], _all_rotated),
}




def _pins(*names):
    """Run pins of the main pin module (each takes the oracle module)."""
    import test_oracle_pins as P

    def run(orc):
        for nm in names:
            fn = getattr(P, nm)
            if nm == "test_adjoint_matches_finite_differences_tiny":
                fn(orc, 0.05, 0)
            elif fn.__code__.co_argcount:
                fn(orc)
            else:
                fn()
    return run


# mistakes in the temporal model, the covariance and the adjoint, caught by
# the pins of the main pin module
MUTATIONS.update({
    "sine amplitude 1% off": ([("const R k = (l / two_pi) * sin_cr(phi);",
                                "const R k = (R(1.01) * l / two_pi) * sin_cr(phi);")],
                              _pins("test_velocity_is_derivative_at_life_peak")),
    "sign in the EWA product": ([("it.T2[c] = it.J00 * W[c] + it.J02 * W[6 + c];",
                                  "it.T2[c] = it.J00 * W[c] - it.J02 * W[6 + c];")],
                                _pins("test_ewa_projection_against_numeric_jacobian")),
    "one rotation entry": ([("Rq[1] = R(2) * (x * y - w * z);", "Rq[1] = R(2) * (x * y + w * z);")],
                           _pins("test_ewa_projection_against_numeric_jacobian")),
    "sign of dL/dB": ([("gg[3] += -c.dx * c.dy * gp;", "gg[3] += c.dx * c.dy * gp;")],
                      _pins("test_adjoint_matches_finite_differences_tiny")),
    "sign in dL/dl": ([("dl += (std::sin(phi) / (2.0 * kPi) - del / it.l * std::cos(phi)) * vg;",
                        "dl += (std::sin(phi) / (2.0 * kPi) + del / it.l * std::cos(phi)) * vg;")],
                      _pins("test_adjoint_matches_finite_differences_tiny")),
})


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_pins_catch_planted_mistakes(orc, tmp_path, name):
    """Each mistake, planted in a copy of the oracle, fails its pin (and the
    unmodified oracle passes the same pin, in the tests above)."""
    edits, pin = MUTATIONS[name]
    src = orc.source_text()
    for old, new in edits:
        assert old in src, old
        src = src.replace(old, new)
    path = orc.build_variant(src, os.path.join(str(tmp_path), "liboracle_variant.so"))
    with orc.use_library(path):
        with pytest.raises(AssertionError):
            pin(orc)
