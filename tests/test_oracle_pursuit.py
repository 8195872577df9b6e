"""Pins of the multi-pursuer single-evader game of Section 3.2 (CPU): the
Hamiltonian against a brute-force max-min over control grids, the capture
datum against a hand-built configuration and its gradient against central
differences."""
import itertools

import numpy as np

from oracle import model


def _problem(n, ae=2.0, ap=1.0, umax=1.0):
    return model.Problem(n=n, ham="pursuit_evasion", ham_p=(ae, ap, umax), datum="capture", datum_p=(1.5,),
                         nu=0.04)


def test_hamiltonian_is_the_max_min_over_controls():
    # 2 pursuers + evader: max over the evader's turn rate, min over the
    # pursuers' joint turn rates, of <p, f(x, u)>, on a grid containing +-u_max
    rng = np.random.default_rng(1)
    pb = _problem(9, ae=2.0, ap=1.0, umax=0.7)
    x = rng.normal(0, 2, (5, 9))
    p = rng.normal(0, 1, (5, 9))
    grid = np.linspace(-0.7, 0.7, 15)
    for q in range(5):
        drift = sum((2.0 if j == 2 else 1.0) * (p[q, 3 * j] * np.cos(x[q, 3 * j + 2])
                                                  + p[q, 3 * j + 1] * np.sin(x[q, 3 * j + 2])) for j in range(3))
        best = -np.inf
        for ue in grid:
            worst = min(p[q, 2] * u1 + p[q, 5] * u2 for u1, u2 in itertools.product(grid, grid))
            best = max(best, drift + p[q, 8] * ue + worst)
        np.testing.assert_allclose(model.hamiltonian(pb, x[q:q + 1], p[q:q + 1])[0], best, rtol=1e-12, atol=1e-12)


def test_capture_datum_on_a_built_configuration():
    pb = _problem(9)
    # pursuers at (4, 0) and (0, -2), evader at the origin: nearest is 2 away
    x = np.array([[4.0, 0.0, 0.3, 0.0, -2.0, 1.0, 0.0, 0.0, -0.5]])
    np.testing.assert_allclose(model.datum(pb, x), [2.0 - 1.5])
    g = model.datum_grad(pb, x)
    np.testing.assert_allclose(g[0], [0, 0, 0, 0, -1, 0, 0, 1, 0])


def test_capture_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    pb = _problem(45)
    x = rng.uniform(-10, 10, (20, 45))
    g = model.datum_grad(pb, x)
    h = 1e-6
    for d in range(45):
        e = np.zeros(45)
        e[d] = h
        fd = (model.datum(pb, x + e) - model.datum(pb, x - e)) / (2 * h)
        np.testing.assert_allclose(g[:, d], fd, atol=1e-6)
