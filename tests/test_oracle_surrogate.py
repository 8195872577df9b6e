"""Pins of the oracle's surrogate-accelerated sweep (CPU only).

The sweep is composed of parts pinned elsewhere (the network's forward pass,
Algorithm 1 with a warm start); these checks pin the composition: what is
warm-started, what decides the fallback, and what replaces a flagged state.
"""
import numpy as np

import workloads
from oracle import estimator, mlp, model, surrogate


def _net(n, width, depth, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    sizes = [n + 1] + [width] * depth + [n + 1]
    layers = [(W * scale, rng.normal(0, 0.05, b.shape)) for W, b in mlp.init_params(sizes, rng)]
    norm = np.stack([np.zeros(n + 1), np.ones(n + 1), np.zeros(n + 1), np.ones(n + 1)])
    return layers, norm


def _problem(n=6):
    w = workloads.C5.resized(n=n, box=workloads.dubins_box(n // 3))
    f = dict(w.problem_fields())
    return w, model.Problem(**f)


def test_no_fallback_is_the_warm_started_picard():
    w, pb = _problem()
    x = workloads.queries(w, Q=64, trial=1).astype(np.float64)
    layers, norm = _net(w.n, 32, 2, 1)
    res = surrogate.sweep(pb, layers, norm, x, 1.0, 512, 2, 1024, 3, tol=1e30)
    v_s, g_s = mlp.value_grad_at(layers, norm, x, 1.0)
    warm = estimator.picard(pb, x, 1.0, 512, 2, tol=1e30, p0=g_s, v0=v_s)
    assert not res.fell_back.any()
    np.testing.assert_array_equal(res.v, warm.v)
    np.testing.assert_array_equal(res.grad, warm.grad)
    # the warm start enters: the first residual is measured from v_S
    assert warm.iters_done == 1
    assert abs(warm.resid_hist[0] - np.linalg.norm(warm.v - v_s) / np.linalg.norm(v_s)) <= 1e-14 * warm.resid_hist[0]


def test_fallback_everywhere_is_the_plain_picard():
    w, pb = _problem()
    x = workloads.queries(w, Q=48, trial=2).astype(np.float64)
    layers, norm = _net(w.n, 32, 2, 2)
    res = surrogate.sweep(pb, layers, norm, x, 1.0, 512, 1, 1024, 3, tol=1e-300)
    plain = estimator.picard(pb, x, 1.0, 1024, 3)
    assert res.fell_back.all()
    np.testing.assert_array_equal(res.v, plain.v)
    np.testing.assert_array_equal(res.grad, plain.grad)


def test_partial_fallback_replaces_exactly_the_flagged_states():
    w, pb = _problem()
    x = workloads.queries(w, Q=80, trial=3).astype(np.float64)
    layers, norm = _net(w.n, 32, 2, 3)
    probe = surrogate.sweep(pb, layers, norm, x, 1.0, 512, 1, 1024, 2, tol=1e30)
    tol = float(np.median(probe.warm.rq))
    res = surrogate.sweep(pb, layers, norm, x, 1.0, 512, 1, 1024, 2, tol=tol)
    fb = res.fell_back
    assert 0 < fb.sum() < len(x)
    np.testing.assert_array_equal(fb, ~(probe.warm.rq <= tol))
    plain = estimator.picard(pb, x, 1.0, 1024, 2)
    np.testing.assert_array_equal(res.v[fb], plain.v[fb])        # common draws: per-state results
    np.testing.assert_array_equal(res.v[~fb], probe.warm.v[~fb])


def test_nan_network_falls_back_everywhere():
    w, pb = _problem()
    x = workloads.queries(w, Q=32, trial=4).astype(np.float64)
    layers, norm = _net(w.n, 32, 2, 4)
    layers[1] = (layers[1][0] * np.nan, layers[1][1])
    res = surrogate.sweep(pb, layers, norm, x, 1.0, 512, 2, 1024, 3, tol=1e-3)
    assert res.fell_back.all() and np.all(np.isfinite(res.v))
    np.testing.assert_array_equal(res.v, estimator.picard(pb, x, 1.0, 1024, 3).v)
