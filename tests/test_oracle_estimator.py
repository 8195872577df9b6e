"""Pins of the oracle's estimators and Picard loop against what the mathematics fixes.

Each check is chosen so that a plausible mistake in the oracle (a dropped
term, a sign, sigma vs sigma^2, delta vs nu, a transposed operand) fails at
least one of them:

* closed forms of the exact Cole-Hopf case H = |p|^2/2 (paper, Section 2.1,
  "Exact case") with quadratic and linear data, evaluated with deterministic
  equal-probability quantile nodes in place of random draws, so that the
  comparison is tight instead of statistical;
* the 1D folded-normal closed form and the 2D Rice-distribution quadrature for
  signed-distance data;
* an independent finite-difference solve of v_t + |v_x|^2/2 = nu v_xx
  (fixes delta = 2 nu);
* exactness of the tilted estimator with the Laplace shift on linear data
  (tilted-proposal corollary: ESS = N, value and control-variate gradient exact
  for every draw);
* the c -> 0 limit (remark on the sign of the coefficient);
* Stein gradient vs a finite difference of the value;
* the N^-1/2 rate of the value error (Section 2.5);
* brute-force max-min evaluation of the game Hamiltonians.
"""
import numpy as np
import pytest
from scipy import integrate, special, stats

from oracle import estimator, model, philox


def quantile_nodes_1d(N1):
    return special.ndtri((np.arange(N1) + 0.5) / N1)


def quantile_grid(n, N1):
    """[n, N1^n] tensor grid of 1D quantile nodes (equal-weight quadrature)."""
    q = quantile_nodes_1d(N1)
    mesh = np.meshgrid(*([q] * n), indexing="ij")
    return np.stack([m.ravel() for m in mesh])


def closed_form_quadratic(x, t, nu):
    """H = |p|^2/2, l = |x|^2/2: v = |x|^2/(2(1+t)) + n nu log(1+t), Dv = x/(1+t)."""
    n = x.shape[1]
    return np.sum(x * x, 1) / (2 * (1 + t)) + n * nu * np.log1p(t), x / (1 + t)


# ---------------------------------------------------------------- exact quadratic case
@pytest.mark.parametrize("tilt_theta", [None, "half", "laplace"])
def test_quadratic_datum_closed_form_quantile_nodes(tilt_theta):
    # the equal-probability quantile rule converges like 1/N1 here (weights
    # peak in the tails when untilted), so N1 = 1500 gives ~1e-4 / ~1e-3.
    nu, t = 0.05, 0.5
    pb = model.Problem(n=2, ham="quadratic", datum="half_sqnorm", nu=nu, tilt=True)
    x = np.array([[0.3, -0.4], [1.0, 0.5], [-0.7, 0.2], [0.0, 0.0]])
    c = model.coefficient(pb, x, x)
    assert np.all(c == 1 / (2 * nu))
    if tilt_theta is None:
        theta = None
    elif tilt_theta == "laplace":
        theta = model.tilt(pb, np.sqrt(pb.delta * t), c, model.datum_grad(pb, x))
        np.testing.assert_allclose(theta, -t * x)
    else:                                           # a non-optimal shift
        theta = -0.5 * t * x
    z = quantile_grid(2, 1500)
    est = estimator.value_grad(pb, x, t, z.shape[1], c, theta, z=z)
    v_ref, g_ref = closed_form_quadratic(x, t, nu)
    np.testing.assert_allclose(est.v, v_ref, rtol=0, atol=1.5e-4)
    np.testing.assert_allclose(est.grad, g_ref, rtol=0, atol=2e-3)
    if tilt_theta == "laplace":                    # near zero-variance proposal
        np.testing.assert_allclose(est.v, v_ref, rtol=0, atol=2e-5)
        np.testing.assert_allclose(est.grad, g_ref, rtol=0, atol=2e-4)


def test_quadratic_datum_mc_within_standard_error():
    nu, t, N = 0.05, 0.5, 1 << 15
    delta = 2 * nu
    pb = model.Problem(n=2, ham="quadratic", datum="half_sqnorm", nu=nu, seed=11)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1.1, 1.1, size=(64, 2))
    est = estimator.value_grad(pb, x, t, N, np.full(64, 1 / delta))
    v_ref, _ = closed_form_quadratic(x, t, nu)
    # second moment ratio of the weights, per dimension, for this datum
    ratio = ((1 + t) ** 2 / (1 + 2 * t)) ** 1 * np.exp(np.sum(x * x, 1) * t / (delta * (1 + t) * (1 + 2 * t)))
    se = delta * np.sqrt((ratio - 1) / N)
    assert np.all(np.abs(est.v - v_ref) < 5 * se)


def test_linear_datum_tilt_is_exact_for_any_draws():
    nu, t, N = 0.01, 1.0, 4096
    a = np.array([0.6, -0.8, 0.3])
    pb = model.Problem(n=3, ham="quadratic", datum="linear", nu=nu, datum_p=(0.25,), datum_aux=a,
                       tilt=True, grad_cv=True, seed=5)
    rng = np.random.default_rng(0)
    x = rng.uniform(-2, 2, size=(16, 3))
    sigma = np.sqrt(pb.delta * t)
    p = model.datum_grad(pb, x)
    c = model.coefficient(pb, x, p)
    theta = model.tilt(pb, sigma, c, p)
    est = estimator.value_grad(pb, x, t, N, c, theta)
    v_ref = x @ a + 0.25 - t * np.dot(a, a) / 2
    np.testing.assert_allclose(est.v, v_ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(est.ess, N, rtol=1e-12)
    np.testing.assert_allclose(est.grad, np.tile(a, (16, 1)), rtol=0, atol=1e-12)
    # without the control variate the gradient carries exactly the Stein noise zbar/(c sigma)
    pb.grad_cv = False
    est2 = estimator.value_grad(pb, x, t, N, c, theta)
    np.testing.assert_allclose(est2.grad, a - est2.zbar / (c[:, None] * sigma), rtol=0, atol=1e-12)


# The deterministic quantile rule is accurate only where the weights are not
# concentrated in the tails of z, i.e. for |c| sigma |Dl| = O(1); those pins
# therefore use nu = 0.25 (c = 2, sigma = 0.5 at t = 0.5).  A mistake in the
# formulas (delta vs nu, sigma vs sigma^2, a sign) still moves the result by
# far more than the tolerances.
def test_linear_datum_untilted_value_matches_hopf_lax():
    nu, t = 0.25, 0.5
    a = np.array([1.0, 0.5])
    pb = model.Problem(n=2, ham="quadratic", datum="linear", nu=nu, datum_p=(-0.5,), datum_aux=a)
    x = np.array([[0.2, 0.1], [-1.0, 1.0]])
    z = quantile_grid(2, 2000)
    est = estimator.value_grad(pb, x, t, z.shape[1], np.full(2, 1 / pb.delta), z=z)
    np.testing.assert_allclose(est.v, x @ a - 0.5 - t * np.dot(a, a) / 2, atol=7e-4)


# ------------------------------------------------------------- signed-distance data
def folded_normal_value(x, t, nu):
    """1D, H = p^2/2, l = |x| - 1: v = -(1/c) log E exp(-c(|Y| - 1)), Y ~ N(x, delta t)."""
    delta = 2 * nu
    c, s = 1 / delta, np.sqrt(delta * t)
    mgf = np.exp(c * c * s * s / 2) * (np.exp(-c * x) * special.ndtr(x / s - c * s)
                                       + np.exp(c * x) * special.ndtr(-x / s - c * s))
    return -(np.log(mgf) + c) / c


def test_1d_abs_datum_closed_form():
    nu, t = 0.25, 0.5
    pb = model.Problem(n=1, ham="quadratic", datum="ball", datum_p=(1, 1.0), nu=nu)
    xs = np.array([-1.5, -0.6, -0.1, 0.0, 0.3, 0.9, 2.0])
    z = quantile_nodes_1d(1 << 18)[None, :]
    est = estimator.value_grad(pb, xs[:, None], t, z.shape[1], np.full(len(xs), 1 / pb.delta), z=z)
    np.testing.assert_allclose(est.v, folded_normal_value(xs, t, nu), atol=2e-5)
    h = 1e-5
    dv = (folded_normal_value(xs + h, t, nu) - folded_normal_value(xs - h, t, nu)) / (2 * h)
    np.testing.assert_allclose(est.grad[:, 0], dv, atol=2e-3)


def fd_viscous_1d(nu, t, xs):
    """Explicit central-difference solve of v_t + v_x^2/2 = nu v_xx, v(0,x) = |x| - 1.

    Independent of the Cole-Hopf transform; domain [-6, 6] with linear
    extrapolation at the ends (far outside the region checked).
    """
    dx = 0.01
    grid = np.arange(-6, 6 + dx / 2, dx)
    v = np.abs(grid) - 1.0
    dt = 0.2 * dx * dx / nu
    steps = int(np.ceil(t / dt))
    dt = t / steps
    for _ in range(steps):
        vx = (v[2:] - v[:-2]) / (2 * dx)
        vxx = (v[2:] - 2 * v[1:-1] + v[:-2]) / (dx * dx)
        v[1:-1] = v[1:-1] + dt * (nu * vxx - 0.5 * vx * vx)
        v[0] = 2 * v[1] - v[2]
        v[-1] = 2 * v[-2] - v[-3]
    return np.interp(xs, grid, v)


@pytest.mark.slow
def test_fd_pde_solve_matches_estimator_1d():
    nu, t = 0.25, 0.5
    xs = np.array([-1.2, -0.4, 0.0, 0.25, 0.8, 1.5])
    pb = model.Problem(n=1, ham="quadratic", datum="ball", datum_p=(1, 1.0), nu=nu)
    z = quantile_nodes_1d(1 << 18)[None, :]
    est = estimator.value_grad(pb, xs[:, None], t, z.shape[1], np.full(len(xs), 1 / pb.delta), z=z)
    np.testing.assert_allclose(est.v, fd_viscous_1d(nu, t, xs), atol=2e-4)


def rice_value(r0, t, nu, R=1.0):
    """2D, H = |p|^2/2, l = |x| - R: E exp(-c(|Y| - R)) with |Y| ~ Rice(r0, sigma)."""
    delta = 2 * nu
    c, s = 1 / delta, np.sqrt(delta * t)
    dist = stats.rice(r0 / s, scale=s)
    lo, hi = max(0.0, r0 - 12 * s), r0 + 12 * s
    val, _ = integrate.quad(lambda r: np.exp(-c * (r - R)) * dist.pdf(r), lo, hi, epsabs=0, epsrel=1e-12, limit=400)
    return -np.log(val) / c


def test_2d_disk_datum_rice_quadrature():
    nu, t = 0.25, 0.5
    pb = model.Problem(n=2, ham="quadratic", datum="ball", datum_p=(2, 1.0), nu=nu)
    x = np.array([[1.2, 0.3], [0.2, -0.5], [0.0, 1.0], [-1.4, -0.9]])
    z = quantile_grid(2, 1000)
    est = estimator.value_grad(pb, x, t, z.shape[1], np.full(len(x), 1 / pb.delta), z=z)
    r0 = np.linalg.norm(x, axis=1)
    v_ref = np.array([rice_value(r, t, nu) for r in r0])
    np.testing.assert_allclose(est.v, v_ref, atol=3e-4)
    h = 1e-4
    dvdr = np.array([(rice_value(r + h, t, nu) - rice_value(r - h, t, nu)) / (2 * h) for r in r0])
    np.testing.assert_allclose(est.grad, (dvdr / r0)[:, None] * x, atol=3e-3)


def fd_viscous_2d_disk(nu, t, pts, dx=0.02, L=3.5):
    """Explicit central-difference solve of v_t + |grad v|^2/2 = nu Lap v,
    v(0, x) = |x| - 1 on [-L, L]^2 (linear extrapolation at the edges, far from
    the points checked); independent of the Cole-Hopf transform.  Returns v and
    grad v at pts [P, 2] by bilinear interpolation of the grid."""
    from scipy.interpolate import RegularGridInterpolator
    g = np.arange(-L, L + dx / 2, dx)
    X, Y = np.meshgrid(g, g, indexing="ij")
    v = np.sqrt(X * X + Y * Y) - 1.0
    dt = 0.2 * dx * dx / nu
    steps = int(np.ceil(t / dt))
    dt = t / steps
    for _ in range(steps):
        c = v[1:-1, 1:-1]
        vx = (v[2:, 1:-1] - v[:-2, 1:-1]) / (2 * dx)
        vy = (v[1:-1, 2:] - v[1:-1, :-2]) / (2 * dx)
        lap = (v[2:, 1:-1] + v[:-2, 1:-1] + v[1:-1, 2:] + v[1:-1, :-2] - 4 * c) / (dx * dx)
        v[1:-1, 1:-1] = c + dt * (nu * lap - 0.5 * (vx * vx + vy * vy))
        v[0, :] = 2 * v[1, :] - v[2, :]
        v[-1, :] = 2 * v[-2, :] - v[-3, :]
        v[:, 0] = 2 * v[:, 1] - v[:, 2]
        v[:, -1] = 2 * v[:, -2] - v[:, -3]
    gx, gy = np.gradient(v, dx, dx)
    interp = [RegularGridInterpolator((g, g), f) for f in (v, gx, gy)]
    return interp[0](pts), np.stack([interp[1](pts), interp[2](pts)], 1)


@pytest.mark.slow
def test_fd_pde_solve_matches_estimator_2d_disk():
    # a brute-force grid solve of the PDE itself in 2D (non-smooth datum at the
    # origin, curved level sets) against the estimator on quantile draws
    nu, t = 0.25, 0.5
    pb = model.Problem(n=2, ham="quadratic", datum="ball", datum_p=(2, 1.0), nu=nu)
    x = np.array([[1.2, 0.3], [0.2, -0.5], [0.0, 1.0], [-1.4, -0.9], [0.05, 0.02]])
    z = quantile_grid(2, 1000)
    est = estimator.value_grad(pb, x, t, z.shape[1], np.full(len(x), 1 / pb.delta), z=z)
    v_fd, g_fd = fd_viscous_2d_disk(nu, t, x)
    # measured 1.2e-4 and 2.9e-4 (grid O(dx^2) and bilinear interpolation); a
    # coefficient off by a factor 2 moves v by 0.12
    np.testing.assert_allclose(est.v, v_fd, atol=5e-4)
    np.testing.assert_allclose(est.grad, g_fd, atol=1.5e-3)


# ----------------------------------------------------------------- limits and invariants
def test_c_to_zero_limit_is_gaussian_mean():
    pb = model.Problem(n=3, ham="zero", datum="min_pair_disks", datum_p=(0.5,), nu=0.01,
                       c_min=1e-9, seed=2)
    rng = np.random.default_rng(4)
    x = rng.uniform(-2, 2, size=(8, 3))
    c = model.coefficient(pb, x, model.datum_grad(pb, x))
    assert np.all(c == 1e-9)
    N, t = 2048, 1.0
    est = estimator.value_grad(pb, x, t, N, c)
    z = philox.crn_table(pb.seed, 0, 0, 3, N)
    y = x[:, None, :] + np.sqrt(pb.delta * t) * z.T[None]
    mean_l = np.mean(model.datum(pb, y), axis=1)
    np.testing.assert_allclose(est.v, mean_l, atol=1e-7)


def test_stein_gradient_matches_fd_of_value():
    nu, t = 0.25, 0.5
    pb = model.Problem(n=2, ham="quadratic", datum="ball", datum_p=(2, 1.0), nu=nu)
    x = np.array([[1.2, 0.3], [0.4, -0.9]])
    z = quantile_grid(2, 900)
    c = np.full(2, 1 / pb.delta)
    est = estimator.value_grad(pb, x, t, z.shape[1], c, z=z)
    h = 1e-3
    fd = np.zeros_like(x)
    for d in range(2):
        e = np.zeros(2)
        e[d] = h
        fd[:, d] = (estimator.value_grad(pb, x + e, t, z.shape[1], c, z=z).v
                    - estimator.value_grad(pb, x - e, t, z.shape[1], c, z=z).v) / (2 * h)
    np.testing.assert_allclose(est.grad, fd, atol=3e-3)


@pytest.mark.slow
def test_value_error_decays_as_inverse_sqrt_n():
    nu, t = 0.05, 0.5
    x = np.array([[0.5, -0.3], [0.2, 0.8]])
    v_ref, _ = closed_form_quadratic(x, t, nu)
    Ns = [1 << k for k in range(8, 15)]
    rms = []
    for N in Ns:
        errs = []
        for seed in range(30):
            pb = model.Problem(n=2, ham="quadratic", datum="half_sqnorm", nu=nu, seed=1000 + seed)
            est = estimator.value_grad(pb, x, t, N, np.full(2, 1 / pb.delta))
            errs.append(est.v - v_ref)
        rms.append(np.sqrt(np.mean(np.square(errs))))
    slope = np.polyfit(np.log(Ns), np.log(rms), 1)[0]
    assert -0.6 < slope < -0.4


def test_tilt_consistency_many_seeds():
    # every shift gives a consistent estimator (tilted-proposal corollary)
    nu, t, N = 0.05, 0.5, 4096
    x = np.array([[0.6, -0.2]])
    v_ref, _ = closed_form_quadratic(x, t, nu)
    for th in ([0.0, 0.0], [0.15, -0.05], [-0.3, 0.1]):
        vs = []
        for seed in range(40):
            pb = model.Problem(n=2, ham="quadratic", datum="half_sqnorm", nu=nu, seed=seed + 77)
            vs.append(estimator.value_grad(pb, x, t, N, np.full(1, 1 / pb.delta), np.array([th])).v[0])
        vs = np.array(vs)
        assert abs(vs.mean() - v_ref[0]) < 5 * vs.std() / np.sqrt(len(vs)) + 1e-4


# ------------------------------------------------------------------- Hamiltonians
def brute_dubins(x, p, s_sign=1.0):
    """max over the evader turn rate, min over the pursuer's, from the relative dynamics."""
    ctrl = np.linspace(-1, 1, 201)
    H = 0.0
    for j in range(len(x) // 3):
        x1, x2, x3 = x[3 * j:3 * j + 3]
        p1, p2, p3 = p[3 * j:3 * j + 3]
        best = -np.inf
        for we in ctrl:
            worst = np.inf
            for wp in ctrl:
                f = np.array([-1 + np.cos(x3) + we * x2, s_sign * np.sin(x3) - we * x1, wp - we])
                worst = min(worst, p1 * f[0] + p2 * f[1] + p3 * f[2])
            best = max(best, worst)
        H += best
    return H


def test_dubins_hamiltonian_brute_force():
    rng = np.random.default_rng(9)
    pb = model.Problem(n=6, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=0.01)
    for _ in range(5):
        x = rng.uniform(-3, 3, 6)
        p = rng.standard_normal(6)
        H = model.hamiltonian(pb, x[None], p[None])[0]
        assert abs(H - brute_dubins(x, p)) < 1e-9
    # the printed variant flips the sign of the p2 sin(x3) term
    pb.ham_p = (-1.0, 1.0, 1.0, 1.0)
    x, p = rng.uniform(-3, 3, 6), rng.standard_normal(6)
    assert abs(model.hamiltonian(pb, x[None], p[None])[0] - brute_dubins(x, p, -1.0)) < 1e-9


def test_double_integrator_hamiltonian_brute_force():
    rng = np.random.default_rng(10)
    pb = model.Problem(n=6, ham="double_integrator", datum="knn_balls", nu=0.02, ham_p=(1.0,))
    dirs = rng.standard_normal((200000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    x, p = rng.standard_normal(6), rng.standard_normal(6)
    brute = p[:3] @ x[3:] + np.max(dirs @ p[3:])
    assert abs(model.hamiltonian(pb, x[None], p[None])[0] - brute) < 1e-3


def test_double_integral_plant_hamiltonian_brute_force():
    """The double integral plant of the appendix: x1' = x2, x2' = u, |u| <= 1,
    the Hamiltonian p1 x1' + p2 x2' minimised by the control (u = -sign p2):
    H = p1 x2 - |p2|.  Brute force over a grid of admissible controls, also at
    u_max = 0.5, and the planar (n = 4) form with a disc of controls."""
    rng = np.random.default_rng(11)
    for umax in (1.0, 0.5):
        pb = model.Problem(n=2, ham="double_integrator", ham_p=(umax, -1.0), datum="ball", datum_p=(2, 0.2),
                           nu=0.04)
        u = np.linspace(-umax, umax, 2001)
        for _ in range(20):
            x, p = rng.standard_normal(2), rng.standard_normal(2)
            brute = np.min(p[0] * x[1] + p[1] * u)
            assert abs(model.hamiltonian(pb, x[None], p[None])[0] - brute) < 1e-12
    # hand value: x = (0.3, -0.5), p = (2, -0.7): 2 * (-0.5) - 0.7 = -1.7
    pb = model.Problem(n=2, ham="double_integrator", ham_p=(1.0, -1.0), datum="ball", datum_p=(2, 0.2), nu=0.04)
    assert model.hamiltonian(pb, np.array([[0.3, -0.5]]), np.array([[2.0, -0.7]]))[0] == pytest.approx(-1.7, abs=1e-15)
    pb4 = model.Problem(n=4, ham="double_integrator", ham_p=(1.0, -1.0), datum="ball", datum_p=(2, 0.2), nu=0.04)
    ang = np.linspace(0, 2 * np.pi, 100001)
    disc = np.stack([np.cos(ang), np.sin(ang)], 1)
    for _ in range(10):
        x, p = rng.standard_normal(4), rng.standard_normal(4)
        brute = p[:2] @ x[2:] + np.min(disc @ p[2:])
        assert abs(model.hamiltonian(pb4, x[None], p[None])[0] - brute) < 1e-8


def test_rockets_hamiltonian_brute_force():
    # -max over u_e of min over u_p of <p, f(x, u_e, u_p)> on control grids
    # that contain the bang-bang corners, with the dynamics rows of the
    # Hamiltonian's definition in the appendix on the game of two rockets
    rng = np.random.default_rng(12)
    a, g, um = 64.0, 32.0, 1.0
    pb = model.Problem(n=3, ham="rockets", datum="ball", datum_p=(2, 1.5), nu=0.04, ham_p=(a, g, um))
    us = np.linspace(-um, um, 41)
    for _ in range(6):
        x = np.array([rng.uniform(-100, 100), rng.uniform(-100, 100), rng.uniform(-np.pi / 2, np.pi / 2)])
        p = rng.standard_normal(3)
        ue, up = np.meshgrid(us, us, indexing="ij")
        f1 = a * np.cos(x[2]) + ue * x[0]
        f2 = a * np.sin(x[2]) + a + up * x[0] - g
        f3 = up - ue
        val = p[0] * f1 + p[1] * f2 + p[2] * f3
        brute = -np.max(np.min(val, axis=1))
        np.testing.assert_allclose(model.hamiltonian(pb, x[None], p[None])[0], brute, rtol=1e-12, atol=1e-9)


def test_murmuration_hamiltonian_planar_part_brute_force():
    # the planar part is -max over the bird's turn rate u_e in [-w_e, w_e] of
    # min over the predator's u_p in [-w_p, w_p] of <p, f> with
    # x1' = v_e - v_p cos x4 - u_e x2, x2' = -v_p sin x4 + u_e x1, x4' = u_e - u_p
    # (the dynamics whose max-min gives the printed terms); the altitude term
    # g_lo |p3| - g_hi |p3| is taken as printed
    rng = np.random.default_rng(14)
    ve, vp, we, wp, glo, ghi = 1.0, 1.2, 0.8, 1.5, -0.3, 0.3
    pb = model.Problem(n=4, ham="murmuration", datum="disc_union", datum_p=(0.6, 7), nu=0.09,
                       ham_p=(ve, vp, we, wp, glo, ghi))
    ue = np.linspace(-we, we, 61)
    up = np.linspace(-wp, wp, 61)
    for _ in range(6):
        x = np.concatenate([rng.uniform(-3, 3, 3), rng.uniform(-np.pi, np.pi, 1)])
        p = rng.standard_normal(4)
        UE, UP = np.meshgrid(ue, up, indexing="ij")
        f1 = ve - vp * np.cos(x[3]) - UE * x[1]
        f2 = -vp * np.sin(x[3]) + UE * x[0]
        f4 = UE - UP
        val = p[0] * f1 + p[1] * f2 + p[3] * f4
        brute = np.max(np.min(val, axis=1)) + (glo - ghi) * abs(p[2])
        np.testing.assert_allclose(model.hamiltonian(pb, x[None], p[None])[0], brute, rtol=1e-12, atol=1e-9)


def test_disc_union_datum_and_gradient():
    cen = np.array([[1.15, 0.0], [0.0, 1.15], [-1.15, 0.0]])
    pb = model.Problem(n=4, ham="murmuration", datum="disc_union", datum_p=(0.6, 3), nu=0.09, datum_aux=cen)
    x = np.array([[1.15, 0.3, 5.0, 1.0], [0.0, 0.0, 0.0, 0.0], [2.0, 1.5, -1.0, 0.3]])
    ell = model.datum(pb, x[:, None, :])[:, 0]
    np.testing.assert_allclose(ell, [0.3 - 0.6, 1.15 - 0.6, np.hypot(0.85, 1.5) - 0.6])
    g = model.datum_grad(pb, x)
    h = 1e-6
    for q in (0, 2):                                      # away from ties: central differences
        for d in range(4):
            e = np.zeros(4)
            e[d] = h
            fd = (model.datum(pb, (x[q] + e)[None, None]) - model.datum(pb, (x[q] - e)[None, None]))[0, 0] / (2 * h)
            assert abs(fd - g[q, d]) < 1e-6
    np.testing.assert_array_equal(g[1], [-1.0, 0.0, 0.0, 0.0])   # equidistant: the first centre wins


def test_coefficient_sign_clip_and_regularisation():
    pb = model.Problem(n=3, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=0.01,
                       eta=0.01, c_min=0.5, c_max=20.0)
    x = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.3], [2.0, 2.0, 2.0]])
    p = np.array([[0.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.3, -0.2, 0.1]])
    H = model.hamiltonian(pb, x, p)
    raw = (2 / pb.delta) * H / (np.sum(p * p, 1) + pb.eta)
    c = model.coefficient(pb, x, p)
    assert c[0] == 0.5                                  # H = 0 -> +c_min
    for ci, ri in zip(c[1:], raw[1:]):
        assert np.sign(ci) == np.sign(ri) and 0.5 <= abs(ci) <= 20.0


def test_tube_coefficient_uses_min_zero_h():
    pb = model.Problem(n=3, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=0.01, tube=True)
    rng = np.random.default_rng(12)
    x = rng.uniform(-3, 3, (200, 3))
    p = rng.normal(size=(200, 3))
    H = model.hamiltonian(pb, x, p)
    c = model.coefficient(pb, x, p)
    assert np.all(c[H > 0] == pb.c_min)                  # min{0, H} = 0 -> +c_min
    pb2 = model.Problem(**{**pb.__dict__, "tube": False})
    np.testing.assert_array_equal(c[H < 0], model.coefficient(pb2, x, p)[H < 0])


# ---------------------------------------------------------------- Picard loop
def test_picard_quadratic_is_fixed_after_one_step_crn():
    pb = model.Problem(n=2, ham="quadratic", datum="ball", datum_p=(2, 1.0), nu=0.05, seed=3)
    rng = np.random.default_rng(5)
    x = rng.uniform(-2, 2, (32, 2))
    res = estimator.picard(pb, x, 0.5, 2048, K=3)
    assert res.iters_done == 3
    assert res.resid_hist[1] == 0.0 and res.resid_hist[2] == 0.0


def test_picard_linear_datum_exact_each_iteration_with_tilt():
    a = np.array([0.3, 0.4, -0.5])
    pb = model.Problem(n=3, ham="quadratic", datum="linear", nu=0.01, datum_p=(0.1,), datum_aux=a,
                       tilt=True, grad_cv=True, seed=8)
    x = np.random.default_rng(6).uniform(-3, 3, (10, 3))
    res = estimator.picard(pb, x, 1.0, 1024, K=4)
    np.testing.assert_allclose(res.v, x @ a + 0.1 - np.dot(a, a) / 2, atol=1e-12)
    np.testing.assert_allclose(res.grad, np.tile(a, (10, 1)), atol=1e-12)


def test_picard_early_exit_and_flags():
    pb = model.Problem(n=2, ham="quadratic", datum="ball", datum_p=(2, 1.0), nu=0.05, seed=3)
    x = np.random.default_rng(5).uniform(-2, 2, (32, 2))
    res = estimator.picard(pb, x, 0.5, 2048, K=5, tol=1e-6)
    assert res.iters_done == 2 and res.resid_hist[-1] == 0.0
    assert not res.flags.any()


# ------------------------------------------- stacked disc pairs: the datum of the Dubins workloads
def _min_pair_disks_brute(y, r):
    """min over pairs j of the planar distance |(y[3j], y[3j+1])| minus r, one state at a time."""
    out = np.empty(len(y))
    for q, yq in enumerate(y):
        best = np.inf
        for j in range(len(yq) // 3):
            d = np.sqrt(yq[3 * j] ** 2 + yq[3 * j + 1] ** 2)
            if d < best:
                best = d
        out[q] = best - r
    return out


@pytest.mark.parametrize("m,r", [(1, 0.5), (5, 0.5), (15, 0.5), (15, 0.0), (4, 2.0)])
def test_min_pair_disks_datum_brute_force(m, r):
    rng = np.random.default_rng(100 + m)
    pb = model.Problem(n=3 * m, ham="dubins_pairs", datum="min_pair_disks", datum_p=(r,), nu=0.01)
    y = np.concatenate([rng.uniform(-3, 3, (300, 3 * m)), rng.normal(0, 0.05, (20, 3 * m))])
    y[:, 2::3] = rng.uniform(-50, 50, (len(y), m))          # headings do not enter the datum
    np.testing.assert_allclose(model.datum(pb, y[:, None, :])[:, 0], _min_pair_disks_brute(y, r), rtol=0,
                               atol=1e-14)
    # the [Q, N, n] layout used by the estimator gives the same values
    np.testing.assert_array_equal(model.datum(pb, y.reshape(16, 20, 3 * m)).ravel(),
                                  model.datum(pb, y[:, None, :])[:, 0])


@pytest.mark.parametrize("m", [1, 3, 15])
def test_min_pair_disks_gradient_central_differences(m):
    rng = np.random.default_rng(200 + m)
    pb = model.Problem(n=3 * m, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=0.01)
    x = rng.uniform(-3, 3, (40, 3 * m))
    g = model.datum_grad(pb, x)
    h = 1e-6
    for q in range(len(x)):
        rho = np.hypot(x[q, 0::3], x[q, 1::3])
        srt = np.sort(rho)
        if m > 1 and srt[1] - srt[0] < 1e-3:
            continue                                      # too close to a tie for a difference quotient
        for d in range(3 * m):
            e = np.zeros(3 * m)
            e[d] = h
            fd = (_min_pair_disks_brute((x[q] + e)[None], 0.5) - _min_pair_disks_brute((x[q] - e)[None], 0.5))[0]
            assert abs(fd / (2 * h) - g[q, d]) < 1e-6, (q, d)
        assert abs(np.linalg.norm(g[q]) - 1.0) < 1e-12         # a distance: unit gradient off the kinks


def test_min_pair_disks_gradient_ties_and_centre():
    pb = model.Problem(n=9, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=0.01)
    x = np.array([
        [3.0, 0.0, 0.1, 1.0, 0.0, 0.2, 0.0, 1.0, 0.3],      # pairs 1 and 2 tie at distance 1: pair 1 wins
        [0.6, 0.8, 0.0, 0.8, 0.6, 0.0, 1.0, 0.0, 0.0],      # all three tie: pair 0 wins
        [2.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 2.0],      # pairs 1 and 2 at the centre: 0 (kink rule)
    ])
    g = model.datum_grad(pb, x)
    np.testing.assert_array_equal(g[0], [0, 0, 0, 1.0, 0, 0, 0, 0, 0])
    np.testing.assert_allclose(g[1], [0.6, 0.8, 0, 0, 0, 0, 0, 0, 0], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(g[2], np.zeros(9))
    np.testing.assert_allclose(model.datum(pb, x[:, None, :])[:, 0], [0.5, 0.5, -0.5], rtol=0, atol=1e-15)


# ------------------------------------------------- the general coefficient branch
def test_general_coefficient_branch_exact_case():
    """H = |p|^2/2 through the general branch with eta = 0 and no clipping is
    exactly 1/delta: the exact reduction the coefficient definition is built
    to reproduce.  A wrong factor (1/delta, |p| for |p|^2) fails here."""
    rng = np.random.default_rng(7)
    for nu in (0.01, 0.05, 0.3):
        p = rng.normal(size=(500, 6)) * rng.uniform(0.1, 10, (500, 1))
        H = 0.5 * np.sum(p * p, axis=1)
        c = model.frozen_coefficient(H, p, 2 * nu, eta=0.0, c_min=0.0, c_max=np.inf)
        np.testing.assert_allclose(c, 1.0 / (2 * nu), rtol=4e-16, atol=0)
    # the regularised denominator: eta = |p|^2 halves it
    p = np.array([[3.0, 4.0]])
    c = model.frozen_coefficient(np.array([12.5]), p, 0.1, eta=25.0, c_min=0.0, c_max=np.inf)
    assert c[0] == pytest.approx(5.0, rel=1e-15)


def test_general_coefficient_clip_keeps_sign():
    p = np.ones((5, 2))
    H = np.array([1e9, -1e9, 1e-12, -1e-12, 0.0])
    c = model.frozen_coefficient(H, p, 0.02, eta=0.0, c_min=0.5, c_max=20.0)
    np.testing.assert_array_equal(c, [20.0, -20.0, 0.5, -0.5, 0.5])


def test_dubins_coefficient_hand_values():
    """One Dubins pair worked by hand (nu = 0.01, so 2/delta = 100; eta = 0.01).

    x = (0, 2, pi/2), p = (1, 0.5, 0.25), unit speeds and turn bound:
      H = p1 (cos x3 - 1) + p2 sin x3 + |p1 x2 - p2 x1 - p3| - |p3|
        = -1 + 0.5 + 1.75 - 0.25 = 1,     |p|^2 + eta = 1.3225,  c = 100 / 1.3225.
    p = (1, -2, 0): H = -1 - 2 + 2 - 0 = -1,  |p|^2 + eta = 5.01,  c = -100 / 5.01;
    with the printed sign of the p2 term (s = -1): H = -1 + 2 + 2 = 3, c = 300 / 5.01;
    with the tube coefficient min{0, H}: H = 0 there, so c = +c_min.
    """
    x = np.array([[0.0, 2.0, np.pi / 2]] * 2)
    p = np.array([[1.0, 0.5, 0.25], [1.0, -2.0, 0.0]])
    kw = dict(n=3, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=0.01, eta=0.01)
    c = model.coefficient(model.Problem(ham_p=(1.0, 1.0, 1.0, 1.0), **kw), x, p)
    np.testing.assert_allclose(c, [100 / 1.3225, -100 / 5.01], rtol=1e-14)
    c = model.coefficient(model.Problem(ham_p=(-1.0, 1.0, 1.0, 1.0), **kw), x, p)
    np.testing.assert_allclose(c[1], 300 / 5.01, rtol=1e-14)
    c = model.coefficient(model.Problem(ham_p=(-1.0, 1.0, 1.0, 1.0), tube=True, **kw), x, p)
    assert c[1] == model.Problem(**kw).c_min


# ------------------------------------------------- warm start of the Picard loop
def test_picard_warm_start_value():
    """The "Fix" step with a given v^(0): v0 = l(x) is the plain start; a v0
    that is already the first iterate of a p-independent problem (H = |p|^2/2,
    no shift) gives a zero first residual and no flags; any other v0 changes
    only the first residual."""
    pb = model.Problem(n=2, ham="quadratic", datum="ball", datum_p=(2, 1.0), nu=0.05, seed=3)
    x = np.random.default_rng(5).uniform(-2, 2, (32, 2))
    base = estimator.picard(pb, x, 0.5, 2048, K=3)
    same = estimator.picard(pb, x, 0.5, 2048, K=3, v0=estimator.datum_at(pb, x))
    np.testing.assert_array_equal(same.v, base.v)
    np.testing.assert_array_equal(same.resid_hist, base.resid_hist)
    first = estimator.picard(pb, x, 0.5, 2048, K=1)
    warm = estimator.picard(pb, x, 0.5, 2048, K=2, tol=1e-12, v0=first.v)
    assert warm.resid_hist[0] == 0.0 and warm.iters_done == 1 and not warm.flags.any()
    v0 = estimator.datum_at(pb, x) + 1.0
    other = estimator.picard(pb, x, 0.5, 2048, K=3, v0=v0)
    np.testing.assert_array_equal(other.v, base.v)
    np.testing.assert_array_equal(other.resid_hist[1:], base.resid_hist[1:])
    assert other.resid_hist[0] == pytest.approx(np.linalg.norm(first.v - v0) / np.linalg.norm(v0), rel=1e-14)


def test_picard_nan_warm_start_is_flagged():
    """A non-finite relative change is not within tolerance: every state with
    a NaN start is flagged and the loop does not stop early on a NaN residual."""
    pb = model.Problem(n=3, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=0.01, tilt=True,
                       seed=4)
    x = np.random.default_rng(9).uniform(-3, 3, (16, 3))
    v0 = np.zeros(16)
    v0[[2, 7]] = np.nan
    res = estimator.picard(pb, x, 1.0, 1024, K=1, tol=1e-3, v0=v0)
    assert res.flags[2] and res.flags[7]
    assert np.isnan(res.resid_hist[0])
    res = estimator.picard(pb, x, 1.0, 1024, K=3, tol=1e-3, v0=v0)
    assert res.iters_done == 3 or res.resid_hist[-1] < 1e-3
