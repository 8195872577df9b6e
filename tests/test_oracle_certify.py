"""Pins of the certification oracle.

* The corollary's guarantee as a property: for any true values and any
  estimate within E of them, no state with v <= 0 is certified SAFE and no
  state with v > 0 is certified UNSAFE; labels change only inside |v_hat| <= E.
* The sampling margin against the exact Cole-Hopf case (H = |p|^2/2,
  l = |x|^2/2 >= 0, so g_min = 0 and g_max = inf; c = 1/delta): over many
  independent draw sets the plain estimator leaves the margin no more often
  than delta_p (Hoeffding is conservative, so far less often), both with the
  true mean and with the estimate's own mean.
* The margin inverts the tail bound: the bound evaluated at the margin
  returns delta_p.
* The c -> 0 limit of the margin is Hoeffding's margin for a mean of values
  in [g_min, g_max].
"""
import numpy as np

from oracle import certify, estimator, model


def test_classification_never_admits_a_wrong_sign():
    rng = np.random.default_rng(0)
    v_true = rng.normal(0, 1, 100000)
    E = 0.3
    v_hat = v_true + rng.uniform(-E, E, v_true.shape)
    lab = certify.classify(v_hat, E)
    assert not np.any((lab == certify.SAFE) & (v_true <= 0))
    assert not np.any((lab == certify.UNSAFE) & (v_true > 0))
    assert np.all(lab[np.abs(v_hat) > E] != certify.UNDETERMINED)
    assert np.all(lab[np.abs(v_hat) <= E] == certify.UNDETERMINED)
    # ties at the margin are undetermined; per-state margins add to E
    np.testing.assert_array_equal(certify.classify([0.3, -0.3, 0.31, 0.5], 0.3, [0, 0, 0, 0.25]), [0, 0, 1, 0])


def test_budget_terms():
    E = certify.error_budget(2.0, 0.5, 3, 1.0, 10000, np.exp(-4.0), 0.01, 0.5, 0.04)
    np.testing.assert_allclose(E, 0.25 + 0.02 + 0.01 + 0.1)


def test_margin_inverts_the_tail_bound():
    c, N, dp = np.array([2.0, -3.0, 0.5]), 4096, 0.05
    v = np.array([0.1, 0.4, -0.2])
    g_min, g_max = -0.5, 1.0
    eps = certify.mc_margin(v, c, N, dp, g_min, g_max)
    assert np.all(np.isfinite(eps))
    e1, e2 = np.exp(-c * g_min), np.exp(-c * g_max)
    alpha, beta = np.minimum(e1, e2), np.maximum(e1, e2)
    mu = np.exp(-c * v)
    tail = 2 * np.exp(-2 * N * mu ** 2 * (1 - np.exp(-np.abs(c) * eps)) ** 2 / (beta - alpha) ** 2)
    np.testing.assert_allclose(tail, dp, rtol=1e-9)
    # a range too wide for N gives no finite margin (r >= 1)
    assert np.isinf(certify.mc_margin(np.array([0.4]), np.array([-3.0]), N, dp, g_min, 3.0)[0])


def test_margin_small_c_limit_is_hoeffding():
    N, dp = 1000, 0.1
    eps = certify.mc_margin(np.array([0.3]), np.array([1e-7]), N, dp, -1.0, 2.0)
    np.testing.assert_allclose(eps, 3.0 * np.sqrt(np.log(2 / dp) / (2 * N)), rtol=1e-5)


def test_margin_covers_the_exact_case():
    nu, t, N, dp = 0.5, 0.5, 256, 0.1
    pb = model.Problem(n=1, ham="quadratic", datum="half_sqnorm", nu=nu, sample_mode="fresh")
    x = np.array([[0.0], [0.6], [1.0]])
    c = np.full(3, 1.0 / pb.delta)
    v_exact = x[:, 0] ** 2 / (2 * (1 + t)) + nu * np.log1p(t)
    eps_true = certify.mc_margin(v_exact, c, N, dp, 0.0, mu=np.exp(-c * v_exact))
    miss_true = miss_hat = 0
    trials = 200
    for s in range(trials):
        est = estimator.value_grad(model.Problem(**{**pb.__dict__, "seed": 1000 + s}), x, t, N, c)
        err = np.abs(est.v - v_exact)
        miss_true += np.sum(err >= eps_true)
        miss_hat += np.sum(err >= certify.mc_margin(est.v, c, N, dp, 0.0))
    assert np.all(np.isfinite(eps_true))
    assert miss_true <= dp * 3 * trials and miss_hat <= dp * 3 * trials
    assert miss_true == 0                       # the bound is far from tight here


def test_bernstein_margin_covers_the_exact_case_and_is_tighter():
    # the same exact case; the empirical Bernstein margin needs the sweep's
    # ESS; it must cover the error at least as often as promised, and it is
    # far narrower than Hoeffding's where the weight range is wide
    nu, t, N, dp = 0.05, 0.5, 2048, 0.1
    pb = model.Problem(n=1, ham="quadratic", datum="half_sqnorm", nu=nu, sample_mode="fresh")
    x = np.array([[0.0], [0.3], [0.6], [1.1]])
    c = np.full(4, 1.0 / pb.delta)
    v_exact = x[:, 0] ** 2 / (2 * (1 + t)) + nu * np.log1p(t)
    miss = 0
    trials = 200
    widths_b, widths_h = [], []
    for s in range(trials):
        est = estimator.value_grad(model.Problem(**{**pb.__dict__, "seed": 5000 + s}), x, t, N, c)
        eb = certify.bernstein_margin(est.v, c, est.ess, N, dp, 0.0)
        miss += np.sum(np.abs(est.v - v_exact) >= eb)
        widths_b.append(eb)
        widths_h.append(certify.mc_margin(est.v, c, N, dp, 0.0))
    assert miss <= dp * 3 * trials
    wb, wh = np.median(widths_b, 0), np.median(widths_h, 0)
    assert np.all(wb < wh)
    # at x = 1.1 the weight range over the mean is ~60: no Hoeffding margin at
    # this N, a finite Bernstein one
    assert np.isinf(wh[3]) and np.isfinite(wb[3])
    # zero variance (ESS = N) and a zero range give a zero margin
    np.testing.assert_array_equal(certify.bernstein_margin([0.2], [1.0], [N], N, dp, 0.5, 0.5), [0.0])
