"""Pins of the marching-squares oracle: a linear field (contour points exact
on the line, total length the line's length inside the grid), a circle
(length within 1 % of 2 pi r, points within a hundredth of a cell of the
circle), and the two saddle cells decided by the cell centre, by hand."""
import numpy as np

from oracle import contour


def test_linear_field_is_exact():
    ny, nx = 20, 30
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    a, b, c = 0.3, -1.0, 7.25                       # the line y = 0.3 x + 7.25
    seg = contour.segments(a * x + b * y + c)
    pts = seg.reshape(-1, 2)
    np.testing.assert_allclose(a * pts[:, 0] + b * pts[:, 1] + c, 0.0, atol=1e-12)
    length = np.sum(np.hypot(seg[:, 2] - seg[:, 0], seg[:, 3] - seg[:, 1]))
    x_end = min((ny - 1 - c) / a, nx - 1.0)          # where the line leaves the grid
    np.testing.assert_allclose(length, np.hypot(x_end, a * x_end), rtol=1e-12)


def test_circle_length_and_radius():
    n, r = 128, 37.3
    y, x = np.mgrid[0:n, 0:n].astype(float)
    seg = contour.segments(np.hypot(x - 64.2, y - 61.7) - r)
    length = np.sum(np.hypot(seg[:, 2] - seg[:, 0], seg[:, 3] - seg[:, 1]))
    assert abs(length - 2 * np.pi * r) < 0.01 * 2 * np.pi * r
    pts = seg.reshape(-1, 2)
    assert np.max(np.abs(np.hypot(pts[:, 0] - 64.2, pts[:, 1] - 61.7) - r)) < 0.01


def test_saddles_by_hand():
    # inside corners c0 and c2 (case 5); centre mean -0.25 <= 0: inside, so the
    # segments cut off the outside corners c1 (edges e0, e1) and c3 (e2, e3)
    v = np.array([[-1.0, 0.5], [0.5, -1.0]])       # rows y = 0, 1; v[0,1] is c1, v[1,0] is c3
    seg = contour.canonical(contour.segments(v))
    t = 1.0 / 1.5
    expect = contour.canonical(np.array([[t, 0.0, 1.0, 1 - t], [0.0, t, 1 - t, 1.0]]))
    np.testing.assert_allclose(seg, expect, atol=1e-12)
    # centre outside (mean 0.25 > 0): the segments cut off the inside corners c0 and c2
    v = np.array([[-0.5, 1.0], [1.0, -0.5]])
    seg = contour.canonical(contour.segments(v))
    t = 0.5 / 1.5
    expect = contour.canonical(np.array([[0.0, t, t, 0.0], [1.0, 1 - t, 1 - t, 1.0]]))
    np.testing.assert_allclose(seg, expect, atol=1e-12)
