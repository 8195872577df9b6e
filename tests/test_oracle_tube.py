"""Pins of the oracle's time-marching step and of the bfloat16-storage network
forward that serves as its datum.

* Semigroup: for H = |p|^2/2 with l = |x|^2/2 the value is known in closed form
  at every time (paper, Section 2.1, exact Cole-Hopf case), so a step from
  t_prev to t_prev + dt whose datum is the closed form at t_prev must return the
  closed form at t_prev + dt (deterministic quantile nodes, tight tolerance).
  A wrong horizon (t_prev + dt instead of dt), a dropped warm start or a datum
  evaluated at the wrong time fails it.
* A step from t_prev = 0 whose datum is the terminal l and whose warm start is
  (l, Dl) is Algorithm 1 itself: bit-identical to the oracle's Picard loop on
  the same draws.
* bfloat16 rounding: hand values at ties, agreement with the independent
  rounding of the draw generator, and the storage forward reduces to the
  plain forward when rounding is the identity.
"""
import numpy as np
import pytest
from scipy import special

from oracle import estimator, mlp, model, philox


def closed_form(x, t, nu):
    n = x.shape[-1]
    return np.sum(x * x, -1) / (2 * (1 + t)) + n * nu * np.log1p(t), x / (1 + t)


def quantile_grid(n, N1):
    q = special.ndtri((np.arange(N1) + 0.5) / N1)
    mesh = np.meshgrid(*([q] * n), indexing="ij")
    return np.stack([m.ravel() for m in mesh])


@pytest.mark.parametrize("t_prev,dt", [(0.25, 0.5), (1.0, 0.1)])
def test_semigroup_step_reproduces_closed_form(t_prev, dt):
    nu = 0.05
    pb = model.Problem(n=2, ham="quadratic", datum="half_sqnorm", nu=nu, tilt=True)
    x = np.array([[0.3, -0.4], [1.0, 0.5], [-0.7, 0.2], [0.0, 0.0], [1.5, -1.2]])
    v0, p0 = closed_form(x, t_prev, nu)
    z = quantile_grid(2, 1500)
    res = estimator.tube_step(pb, x, t_prev, dt, z.shape[1], 2,
                              lambda y: closed_form(y, t_prev, nu)[0], v0, p0, z=z)
    v_ref, g_ref = closed_form(x, t_prev + dt, nu)
    # Laplace shift from the exact gradient: near zero-variance proposal
    np.testing.assert_allclose(res.v, v_ref, rtol=0, atol=2e-5)
    np.testing.assert_allclose(res.grad, g_ref, rtol=0, atol=3e-4)
    # the one-step horizon is dt, not t_prev + dt
    wrong = estimator.tube_step(pb, x, t_prev, t_prev + dt, z.shape[1], 1,
                                lambda y: closed_form(y, t_prev, nu)[0], v0, p0, z=z)
    assert np.max(np.abs(wrong.v - v_ref)) > 1e-3


def test_step_from_terminal_datum_is_algorithm_1():
    pb = model.Problem(n=3, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=0.01,
                       ham_p=(1.0, 1.0, 1.0, 1.0), tilt=True, tube=True, seed=77, problem_id=3)
    rng = np.random.default_rng(5)
    x = np.column_stack([rng.uniform(-2, 2, 40), rng.uniform(-2, 2, 40), rng.uniform(-np.pi, np.pi, 40)])
    dt, N, K = 0.3, 2048, 3
    ref = estimator.picard(pb, x, dt, N, K, time_step=4)
    res = estimator.tube_step(pb, x, 0.0, dt, N, K, lambda y: model.datum(pb, y),
                              estimator.datum_at(pb, x), model.datum_grad(pb, x), time_step=4)
    assert np.array_equal(res.v, ref.v) and np.array_equal(res.grad, ref.grad)
    assert np.array_equal(res.resid_hist, ref.resid_hist)


def test_round_bf16_ties_and_agreement_with_draw_rounding():
    r = mlp.round_bf16(np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -30, -2.5, 3.0 * 2 ** -20]))
    np.testing.assert_array_equal(r, [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 3.0 * 2 ** -20])
    a = np.random.default_rng(1).normal(0, 10, 200000).astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(mlp.round_bf16(a), philox.round_bf16(a))


def test_storage_forward_reduces_to_plain_forward(monkeypatch):
    rng = np.random.default_rng(2)
    params = mlp.init_params([4, 16, 16, 4], rng)
    X = rng.normal(size=(50, 4))
    plain, _ = mlp.forward(params, X)
    monkeypatch.setattr(mlp, "round_bf16", lambda a: np.asarray(a, dtype=np.float64))
    np.testing.assert_array_equal(mlp.forward_bf16_storage(params, X), plain)


def test_storage_forward_within_bf16_bound_and_value_head():
    rng = np.random.default_rng(3)
    params = mlp.init_params([4, 32, 32, 4], rng)
    norm = np.stack([rng.normal(0, 0.3, 4), rng.uniform(0.5, 2, 4), rng.normal(0, 0.3, 4), rng.uniform(0.5, 2, 4)])
    y = rng.normal(size=(7, 9, 3))
    v = mlp.value_at(params, norm, y, 0.4)
    assert v.shape == (7, 9)
    full = mlp.predict(params, np.concatenate([y.reshape(-1, 3), np.full((63, 1), 0.4)], 1), *norm)
    # three roundings of relative size 2^-9 along the path
    assert np.max(np.abs(v.ravel() - full[:, 0])) <= 0.05 * np.max(np.abs(full[:, 0]))
    v2, g2 = mlp.value_grad_at(params, norm, y.reshape(-1, 3), 0.4)
    np.testing.assert_array_equal(v2, v.ravel())
    assert g2.shape == (63, 3)
