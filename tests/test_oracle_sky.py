"""Pins of the oracle's sky composite (Sec. 3.4, sky refinement:
C_f = C + (1 - O) f_sky(d) with a learnable cube map f_sky): a constant cube
map reduces to a constant background; the six axis directions land on the
six face centres; directions on either side of every cube edge land on the
facing edges of the two faces (the face orientations fit together); the
composite is linear in the cube map and the opacity; and the adjoint matches
finite differences."""
import numpy as np
import pytest

import gen


@pytest.fixture(scope="module")
def cam():
    return gen.yaw_camera(48, 32, 30.0, (0.0, 0.0, 0.0))


def test_constant_cube_is_a_background(orc, cam):
    rng = np.random.default_rng(0)
    H, W = cam["height"], cam["width"]
    img, opac = rng.random((3, H, W)), rng.random((H, W))
    cube = np.empty((6, 3, 8, 8))
    cube[:, 0], cube[:, 1], cube[:, 2] = 0.25, 0.5, 0.75
    out = orc.sky_f64(img, opac, cube, cam)
    ref = img + (1.0 - opac)[None] * np.array([0.25, 0.5, 0.75])[:, None, None]
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-6)  # bilinear weights are FP32 (their sum is 1 to rounding)


def test_axis_directions_hit_face_centres(orc):
    axes = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    for f, d in enumerate(axes):
        face, uv = orc.sky_face_uv(np.array(d, np.float64))
        assert face == f and np.allclose(uv, 0.5), (d, face, uv)


def _edge_uv(face, uv):
    """Which edge of the face a boundary point lies on: (side, coordinate along it)."""
    u, v = uv
    if abs(u) < 1e-4:
        return "u0", v
    if abs(u - 1) < 1e-4:
        return "u1", v
    if abs(v) < 1e-4:
        return "v0", u
    if abs(v - 1) < 1e-4:
        return "v1", u
    return None, None


def test_faces_meet_along_their_edges(orc):
    """For each of the 12 cube edges, points a hair to either side map to
    the boundary of their two faces, and moving along the edge moves both
    face coordinates monotonically: neighbouring faces are not mirrored or
    turned against each other."""
    eps = 1e-5  # the face and coordinates are taken in FP32
    checked = 0
    for a in range(3):
        for b in range(a + 1, 3):
            c = 3 - a - b
            for sa in (1, -1):
                for sb in (1, -1):
                    tracks = {0: [], 1: []}
                    for s in np.linspace(-0.8, 0.8, 5):
                        for side, (ka, kb) in enumerate(((1.0, 1.0 - eps), (1.0 - eps, 1.0))):
                            d = np.zeros(3)
                            d[a], d[b], d[c] = sa * ka, sb * kb, s
                            face, uv = orc.sky_face_uv(d)
                            edge, along = _edge_uv(face, uv)
                            assert edge is not None, (d, face, uv)
                            tracks[side].append((face, edge, along))
                    for side in (0, 1):
                        faces = {t[0] for t in tracks[side]}
                        edges = {t[1] for t in tracks[side]}
                        assert len(faces) == 1 and len(edges) == 1, tracks[side]
                        along = np.array([t[2] for t in tracks[side]])
                        assert np.all(np.diff(along) > 0) or np.all(np.diff(along) < 0)
                    assert tracks[0][0][0] != tracks[1][0][0]
                    # the two faces see the same point of the edge at the same place (up to direction)
                    p0 = np.array([t[2] for t in tracks[0]])
                    p1 = np.array([t[2] for t in tracks[1]])
                    assert np.allclose(p0, p1, atol=1e-4) or np.allclose(p0, 1 - p1, atol=1e-4)
                    checked += 1
    assert checked == 12


def test_linear_and_adjoint_matches_finite_differences(orc, cam):
    rng = np.random.default_rng(1)
    H, W = cam["height"], cam["width"]
    R = 6
    img, opac = rng.random((3, H, W)), rng.random((H, W))
    c1, c2 = rng.random((6, 3, R, R)), rng.random((6, 3, R, R))
    jit = (rng.random((2, H, W)) - 0.5).astype(np.float32)
    o1 = orc.sky_f64(img, opac, c1, cam, jit) - img
    o2 = orc.sky_f64(img, opac, c2, cam, jit) - img
    o12 = orc.sky_f64(img, opac, 2 * c1 - 3 * c2, cam, jit) - img
    np.testing.assert_allclose(o12, 2 * o1 - 3 * o2, atol=1e-12)
    g = rng.standard_normal((3, H, W))
    dO, dC = orc.sky_bwd_f64(g, opac, c1, cam, jit)
    L = lambda cube, op: float(np.sum(g * orc.sky_f64(img, op, cube, cam, jit)))  # noqa: E731
    h = 1e-6
    touched = np.argwhere(np.abs(dC) > 0)
    assert len(touched) > 50
    for idx in touched[rng.choice(len(touched), 40, replace=False)]:
        cp, cm = c1.copy(), c1.copy()
        cp[tuple(idx)] += h
        cm[tuple(idx)] -= h
        fd = (L(cp, opac) - L(cm, opac)) / (2 * h)
        assert abs(fd - dC[tuple(idx)]) <= 1e-7 * max(1.0, abs(fd)), (idx, fd, dC[tuple(idx)])
    for _ in range(20):
        y, x = rng.integers(0, H), rng.integers(0, W)
        op, om = opac.copy(), opac.copy()
        op[y, x] += h
        om[y, x] -= h
        fd = (L(c1, op) - L(c1, om)) / (2 * h)
        assert abs(fd - dO[y, x]) <= 1e-7 * max(1.0, abs(fd))
