"""Large sizes on the device (64-bit offsets, many splits, long sample
streams) against the FP64 oracle on sampled states."""
import numpy as np
import pytest

import workloads
from oracle import estimator, model
from tests._helpers import gpu_problem, grad_tol, oracle_problem, to_dev, value_tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2605_18566_amd import Context
    c = Context(0)
    yield c
    c.close()


def _check(name, v, g, ref, c, theta, sigma, N):
    vt = value_tol(ref.v, c, theta, sigma, ref.lmax)
    dv = np.abs(v - ref.v)
    dg = np.linalg.norm(g - ref.grad, axis=1)
    gt = grad_tol(ref.grad, c, sigma, N)
    print(f"[{name}] worst |dv|/tol {np.max(dv / vt):.3f}, worst |dgrad|/tol {np.max(dg / gt):.3f}", flush=True)
    assert np.all(dv <= vt) and np.all(dg <= gt)


def test_long_sample_stream(ctx):
    # N = 2^22 common draws (a 4M-sample float32 table, many sample splits)
    from paper_2605_18566_amd import value_grad
    fields = dict(workloads.C2.problem_fields())
    N, Q, t = 1 << 22, 64, 0.5
    x = workloads.queries(workloads.C2, Q=Q, trial=21).astype(np.float64)
    pb = oracle_problem(fields)
    sigma = np.sqrt(pb.delta * t)
    p = model.datum_grad(pb, x)
    c = model.coefficient(pb, x, p).astype(np.float32).astype(np.float64)
    theta = model.tilt(pb, sigma, c, p).astype(np.float32).astype(np.float64)
    v, g, _ = value_grad(ctx, gpu_problem(fields), to_dev(np.ascontiguousarray(x.T)), t, N, to_dev(c),
                         to_dev(np.ascontiguousarray(theta.T)))
    v, g = v.cpu().numpy(), g.cpu().numpy().T
    sel = np.arange(0, Q, 8)
    ref = estimator.value_grad(pb, x[sel], t, N, c[sel], theta[sel])
    _check("N = 2^22", v[sel], g[sel], ref, c[sel], theta[sel], sigma, N)


def test_many_states(ctx):
    # Q = 2^23 states (n = 3: a 100 MB state array, 64-bit element offsets)
    from paper_2605_18566_amd import value_grad
    fields = dict(workloads.C2.problem_fields())
    N, Q, t = 512, 1 << 23, 0.3
    x = workloads.queries(workloads.C2, Q=Q, trial=22)
    pb = oracle_problem(fields)
    sigma = np.sqrt(pb.delta * t)
    c = np.full(Q, 0.5, dtype=np.float32)
    xd = to_dev(np.ascontiguousarray(x.T))
    v, g, _ = value_grad(ctx, gpu_problem(fields), xd, t, N, to_dev(c), None)
    sel = np.concatenate([np.arange(8), Q - 1 - np.arange(8), np.random.default_rng(3).choice(Q, 16)])
    v, g = v.cpu().numpy()[sel], g.cpu().numpy()[:, sel].T
    cs = c[sel].astype(np.float64)
    ref = estimator.value_grad(pb, x[sel].astype(np.float64), t, N, cs)
    _check("Q = 2^23", v, g, ref, cs, np.zeros((len(sel), 3)), sigma, N)
