"""Pins of the FP64 surrogate-network reference: its gradients against central
finite differences of its own loss (tiny net), and the closed form of the
SiLU derivative."""
import numpy as np

from oracle import mlp


def test_dsilu_matches_finite_difference():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    np.testing.assert_allclose(mlp.dsilu(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), atol=1e-8)


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [5, 7, 6, 5]
    params = mlp.init_params(sizes, rng)
    params = [(W, rng.normal(0, 0.1, b.shape)) for W, b in params]
    X = rng.normal(size=(9, 5))
    T = rng.normal(size=(9, 5))
    lam = 0.7
    loss, grads = mlp.loss_and_grads(params, X, T, lam)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            it = np.nditer(arr, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = arr[idx]
                arr[idx] = old + h
                lp, _ = mlp.loss_and_grads(params, X, T, lam)
                arr[idx] = old - h
                lm, _ = mlp.loss_and_grads(params, X, T, lam)
                arr[idx] = old
                assert abs((lp - lm) / (2 * h) - g[idx]) < 1e-6 * max(1.0, abs(g[idx]))


def test_loss_weights_value_and_gradient_outputs():
    params = [(np.zeros((3, 2)), np.array([1.0, 2.0, 3.0]))]
    X = np.zeros((4, 2))
    T = np.zeros((4, 3))
    loss, _ = mlp.loss_and_grads(params, X, T, lam=0.5)
    # (1^2) + (0.5/2)(2^2 + 3^2)
    assert np.isclose(loss, 1.0 + 0.25 * 13.0)
