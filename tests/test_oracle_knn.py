"""Pins of the brute-force nearest-neighbour oracle (CPU)."""
import itertools

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import knn


def test_matches_a_kd_tree_on_random_points():
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 10, (2000, 3)).astype(np.float32)
    got = knn.knn(pos, 7)
    d, j = cKDTree(pos.astype(np.float64)).query(pos.astype(np.float64), k=8)
    # continuous random points: no ties, so the sets and orders agree
    np.testing.assert_array_equal(got, j[:, 1:])
    d_ours = np.sqrt(knn.dist2_f32(pos[:, None, :], pos[got]).astype(np.float64))
    np.testing.assert_allclose(d_ours, d[:, 1:], rtol=1e-6)


def test_lattice_closed_form_and_ties_by_index():
    # unit lattice 6 x 6 x 6: an interior point has 6 face neighbours at
    # distance 1, then 12 edge neighbours at sqrt 2 of which the lowest index wins
    g = np.array(list(itertools.product(range(6), repeat=3)), dtype=np.float32)   # index = 36 x + 6 y + z
    i = 36 * 2 + 6 * 3 + 2
    nb = knn.knn(g, 7, queries=[i])[0]
    faces = sorted([i - 36, i + 36, i - 6, i + 6, i - 1, i + 1])
    assert sorted(nb[:6].tolist()) == faces
    assert list(nb[:6]) == faces                       # equal distances: ascending index
    edges = [i + 36 * a + 6 * b + c for a, b, c in itertools.product((-1, 0, 1), repeat=3)
             if abs(a) + abs(b) + abs(c) == 2]
    assert nb[6] == min(edges)


def test_duplicates_and_self_exclusion():
    pos = np.zeros((10, 3), dtype=np.float32)
    pos[7] = 1.0
    nb = knn.knn(pos, 3)
    assert list(nb[0]) == [1, 2, 3] and list(nb[4]) == [0, 1, 2]
    assert list(nb[7]) == [0, 1, 2]
    with pytest.raises(ValueError):
        knn.knn(pos, 10)


def test_float32_rounding_decides_near_ties():
    # two neighbours whose float64 distances differ but float32 ones are equal:
    # the lower index wins, as the float32 rule says
    a = np.array([[0, 0, 0], [1, 0, 0], [0, 1.0000000001, 0]], dtype=np.float32)
    assert list(knn.knn(a, 2, queries=[0])[0]) == [1, 2]
    b = a.copy()
    b[2, 1] = np.nextafter(np.float32(1), np.float32(0))
    assert list(knn.knn(b, 2, queries=[0])[0]) == [2, 1]
