"""Pins of the SSIM oracle: S(x, x) = 1 everywhere; for constant images a
and b the interior value (2ab + C1) / (a^2 + b^2 + C1); symmetry in x and
y; the window is the normalised outer product of the 1D Gaussian; finite
differences of sum g S against the adjoint, border pixels included."""
import numpy as np

from oracle import ssim as os_


def test_identity_and_symmetry():
    rng = np.random.default_rng(0)
    x = rng.random((3, 20, 27))
    y = rng.random((3, 20, 27))
    np.testing.assert_allclose(os_.ssim_map(x, x), 1.0, atol=1e-12)
    np.testing.assert_allclose(os_.ssim_map(x, y), os_.ssim_map(y, x), atol=1e-14)
    assert os_.ssim_map(x, y).max() < 1.0


def test_constant_images_closed_form():
    a, b = 0.3, 0.7
    x = np.full((1, 24, 24), a)
    y = np.full((1, 24, 24), b)
    S = os_.ssim_map(x, y)[0, 5:-5, 5:-5]
    np.testing.assert_allclose(S, (2 * a * b + os_.C1) / (a * a + b * b + os_.C1), rtol=1e-9)


def test_window():
    w = os_.window()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    g = w.sum(axis=1)
    np.testing.assert_allclose(w, np.outer(g, g), rtol=1e-12)
    np.testing.assert_allclose(g[5] / g[6], np.exp(1.0 / (2 * 1.5 ** 2)), rtol=1e-12)


def test_adjoint_matches_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.random((2, 16, 19))
    y = rng.random((2, 16, 19))
    g = rng.standard_normal((2, 16, 19))
    dx = os_.ssim_grad(x, y, g)
    for c, i, j in [(0, 0, 0), (0, 3, 7), (1, 15, 18), (1, 8, 0), (0, 10, 10), (1, 5, 17)]:
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[c, i, j] += h
        xm[c, i, j] -= h
        fd = (np.sum(g * os_.ssim_map(xp, y)) - np.sum(g * os_.ssim_map(xm, y))) / (2 * h)
        assert abs(fd - dx[c, i, j]) <= 1e-6 * max(1.0, abs(dx[c, i, j])), (c, i, j, fd, dx[c, i, j])
