"""Pins of the oracle's reach-avoid projection (oracle/avoid.py).

What fixes it independently of its own code: the reach-avoid property (no
state of the avoid set ever has a value <= 0, whatever the unconstrained
value), the lattice property of the maximum (the result is the smallest value
above both the unconstrained value and the obstacle, and equals one of them),
the obstacle level against a brute-force distance loop, the reported gradient
against central differences of the projected field, idempotence, and the
identity where the obstacle is far away.
"""
import math

import numpy as np

from oracle import avoid, model


def disc_obstacle(n, centres, r):
    return model.Problem(n=n, ham="quadratic", datum="disc_union", datum_p=(r, len(centres)),
                         datum_aux=np.asarray(centres, dtype=np.float64).ravel(), nu=0.05)


CENTRES = [(1.5, 0.0), (-0.5, 1.2), (0.3, -1.4)]


def brute_level(x, centres, r):
    out = np.empty(x.shape[0])
    for q in range(x.shape[0]):
        best = math.inf
        for c0, c1 in centres:
            best = min(best, math.hypot(x[q, 0] - c0, x[q, 1] - c1))
        out[q] = best - r
    return out


def test_obstacle_level_is_the_distance_to_the_discs():
    rng = np.random.default_rng(1)
    x = rng.uniform(-3, 3, (500, 3))
    pb = disc_obstacle(3, CENTRES, 0.6)
    lv, dl = avoid.obstacle_level(pb, x)
    np.testing.assert_allclose(lv, brute_level(x, CENTRES, 0.6), rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(dl, axis=1), 1.0, atol=1e-12)   # a distance has unit slope
    assert np.all(dl[:, 2] == 0.0)                                             # heading does not enter


def test_states_of_the_avoid_set_never_reach():
    rng = np.random.default_rng(2)
    x = rng.uniform(-3, 3, (4000, 3))
    v = rng.uniform(-5, 5, 4000)
    pb = disc_obstacle(3, CENTRES, 0.6)
    vo, _, act = avoid.project(pb, x, v)
    inside = brute_level(x, CENTRES, 0.6) < 0
    assert inside.sum() > 100
    assert np.all(vo[inside] > 0)                          # never counted as reached
    h = -brute_level(x, CENTRES, 0.6)
    assert np.all(vo >= v) and np.all(vo >= h - 1e-12)     # above both
    assert np.all((vo == v) | (np.abs(vo - h) <= 1e-12))   # and equal to one of them
    assert np.array_equal(act, h > v)
    # reached states outside the obstacle's reach keep their value
    keep = (v > h)
    assert np.array_equal(vo[keep], v[keep])


def test_projected_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    n = 3
    a = np.array([0.7, -0.4, 0.25])
    b = -0.9
    x = rng.uniform(-3, 3, (600, n))
    pb = disc_obstacle(n, CENTRES, 0.6)

    def field(xx):
        vo, go, act = avoid.project(pb, xx, xx @ a + b, np.broadcast_to(a, xx.shape).copy())
        return vo, go, act

    v0, g0, act = field(x)
    h = -brute_level(x, CENTRES, 0.6)
    # keep states clear of the projection's kink and of the discs' medial axes
    d = np.sort(np.stack([np.hypot(x[:, 0] - c0, x[:, 1] - c1) for c0, c1 in CENTRES], 1), 1)
    clear = (np.abs(h - (x @ a + b)) > 1e-3) & (d[:, 1] - d[:, 0] > 1e-3) & (d[:, 0] > 1e-3)
    assert clear.sum() > 400 and act[clear].sum() > 50 and (~act[clear]).sum() > 50
    eps = 1e-6
    fd = np.zeros_like(x)
    for k in range(n):
        e = np.zeros(n)
        e[k] = eps
        fd[:, k] = (field(x + e)[0] - field(x - e)[0]) / (2 * eps)
    np.testing.assert_allclose(g0[clear], fd[clear], rtol=0, atol=1e-6)
    # the obstacle branch points away from the nearest centre (ascent of -l_A inward)
    on = clear & act
    nearest = np.argmin(np.stack([np.hypot(x[:, 0] - c0, x[:, 1] - c1) for c0, c1 in CENTRES], 1), 1)
    cen = np.asarray(CENTRES)[nearest]
    assert np.all(np.sum(g0[on, :2] * (x[on, :2] - cen[on]), axis=1) < 0)


def test_idempotent_and_identity_far_away():
    rng = np.random.default_rng(4)
    x = rng.uniform(-3, 3, (1000, 3))
    v = rng.uniform(-5, 5, 1000)
    g = rng.normal(size=(1000, 3))
    pb = disc_obstacle(3, CENTRES, 0.6)
    v1, g1, _ = avoid.project(pb, x, v, g)
    v2, g2, act2 = avoid.project(pb, x, v1, g1)
    assert not act2.any()
    assert np.array_equal(v1, v2) and np.array_equal(g1, g2)
    far = disc_obstacle(3, [(100.0, 100.0)], 0.6)
    v3, g3, act3 = avoid.project(far, x, v, g)
    assert not act3.any() and np.array_equal(v3, v) and np.array_equal(g3, g)


def test_ball_and_knn_obstacles():
    rng = np.random.default_rng(5)
    x = rng.uniform(-2, 2, (300, 6))
    v = np.full(300, -1.0)
    ball = model.Problem(n=6, ham="quadratic", datum="ball", datum_p=(3, 1.0), nu=0.05)
    vo, go, act = avoid.project(ball, x, v, np.zeros((300, 6)))
    rho = np.linalg.norm(x[:, :3], axis=1)
    assert np.array_equal(act, 1.0 - rho > -1.0)
    np.testing.assert_allclose(vo[act], 1.0 - rho[act], atol=1e-12)
    np.testing.assert_allclose(go[act, :3], -x[act, :3] / rho[act, None], atol=1e-12)
    # knn obstacle: per-state neighbour lists
    nb = rng.uniform(-2, 2, (300, 4, 3))
    knn = model.Problem(n=6, ham="double_integrator", ham_p=(1.0,), datum="knn_balls", datum_p=(0.3, 4), nu=0.02)
    lv, _ = avoid.obstacle_level(knn, x, nb)
    ref = np.array([min(np.linalg.norm(x[q, :3] - nb[q, j]) for j in range(4)) - 0.3 for q in range(300)])
    np.testing.assert_allclose(lv, ref, atol=1e-12)
