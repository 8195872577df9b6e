"""The murmuration plug-ins on an MI355X: the flock Hamiltonian and the
union-of-capture-discs datum against the oracle (one frozen sweep with fresh
and common draws, with and without the shift; the Picard loop), and the
slice smoothing against scipy's Gaussian filter (the routine the paper's
topology procedure relies on)."""
import numpy as np
import pytest
from scipy import ndimage

import workloads
from oracle import estimator, model
from tests._helpers import ESS_RTOL_CAP, ess_rtol, gpu_problem, grad_tol, oracle_problem, soa, to_dev, value_tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2605_18566_amd import Context
    c = Context(0)
    yield c
    c.close()


CEN = workloads.murmuration_centres()


@pytest.mark.parametrize("mode,tilt,Q,N", [("fresh", False, 700, 1600), ("crn_step", True, 513, 2000 + 7),
                                           ("fresh", True, 300, 999)])
def test_one_sweep_matches_oracle(ctx, mode, tilt, Q, N):
    from paper_2605_18566_amd import value_grad
    w = workloads.C8
    fields = dict(w.problem_fields(), sample_mode=mode, tilt=tilt)
    x = workloads.queries(w.resized(box=((-2.0, 2.0), (-2.0, 2.0), (-0.5, 0.5), (-np.pi, np.pi))), Q=Q,
                          trial=9).astype(np.float64)
    pb = oracle_problem(fields, aux=CEN.astype(np.float64))
    t = 0.6
    sigma = np.sqrt(pb.delta * t)
    p = model.datum_grad(pb, x)
    c = model.coefficient(pb, x, p).astype(np.float32).astype(np.float64)
    theta = model.tilt(pb, sigma, c, p).astype(np.float32).astype(np.float64)
    ref = estimator.value_grad(pb, x, t, N, c, theta if tilt else None, time_step=3, iteration=2)
    aux = to_dev(CEN.ravel())
    v, g, ess = value_grad(ctx, gpu_problem(fields, aux=aux), to_dev(soa(x)), t, N, to_dev(c),
                           to_dev(soa(theta)) if tilt else None, time_step=3, iteration=2, check_finite=True)
    v, g, ess = (a.cpu().numpy().astype(np.float64) for a in (v, g, ess))
    g = g.T
    th = theta if tilt else np.zeros_like(x)
    vt = value_tol(ref.v, c, th, sigma, ref.lmax)
    assert np.all(np.abs(v - ref.v) <= vt), f"value ratio {np.max(np.abs(v - ref.v) / vt):.2f}"
    assert np.all(np.linalg.norm(g - ref.grad, axis=1) <= grad_tol(ref.grad, c, sigma, N))
    et = ess_rtol(c, th if tilt else None, sigma, ref.lmax)
    held = et <= ESS_RTOL_CAP
    assert held.mean() >= 0.6
    assert np.all((np.abs(ess - ref.ess) <= et * ref.ess)[held])


def test_picard_matches_oracle(ctx):
    from paper_2605_18566_amd import picard_sweep
    w = workloads.C8
    fields = dict(w.problem_fields(), sample_mode="crn_step")
    x = workloads.queries(w, Q=400, trial=11).astype(np.float64)
    pb = oracle_problem(fields, aux=CEN.astype(np.float64))
    out = picard_sweep(ctx, gpu_problem(fields, aux=to_dev(CEN.ravel())), to_dev(soa(x)), 1.0, 1600, 4,
                       time_step=5)
    ref = estimator.picard(pb, x, 1.0, 1600, 4, time_step=5)
    v = out.v.cpu().numpy()
    vt = value_tol(ref.v, ref.c, np.zeros_like(x), np.sqrt(pb.delta), ref.lmax)
    assert np.mean(np.abs(v - ref.v) <= 10 * vt) >= 0.995
    np.testing.assert_allclose(out.resid_hist, ref.resid_hist, rtol=1e-3, atol=1e-6)


@pytest.mark.parametrize("ny,nx,sigma", [(128, 128, 1.5), (37, 53, 1.0), (8, 100, 3.0), (3, 3, 1.5)])
def test_smoothing_matches_scipy(ny, nx, sigma):
    from paper_2605_18566_amd import smooth_slices
    rng = np.random.default_rng(ny * nx)
    v = rng.normal(0, 1, (4, ny, nx)).astype(np.float32)
    got = smooth_slices(to_dev(v), sigma).cpu().numpy()
    ref = np.stack([ndimage.gaussian_filter(s.astype(np.float64), sigma, mode="reflect", truncate=4.0) for s in v])
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-6)
