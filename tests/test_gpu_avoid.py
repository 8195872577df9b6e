"""Reach-avoid obstacle projection (hjg_avoid_project) against the oracle's, on
an MI355X, and one reach-avoid time step (Algorithm 1 then the projection)
against the oracle's step on the same draws.

Tolerance.  The device evaluates the obstacle level in float32 (a few
roundings of the coordinates' scale: sums of n squares or products, one
square root), the oracle in float64, so the lifted value agrees to
2e-6 (1 + |l_A| + s) with s the level's term scale (sum |a_i x_i| + |b| for a
linear level).  The replace-or-keep decision is compared only where the
oracle's margin |(-l_A) - v| exceeds that tolerance (both results are valid
inside it); gradients of replaced states are compared where the nearest
branch of a minimum-type level is unique by a margin (elsewhere the device may
take the other branch, which is also a valid gradient, checked as a unit
vector); states that are kept are bit-identical to the input.
"""
import numpy as np
import pytest

import workloads
from oracle import avoid, estimator
from tests._helpers import gpu_problem, oracle_problem, soa, to_dev, value_tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2605_18566_amd import Context
    c = Context(0)
    yield c
    c.close()


Q_RAGGED = 3 * 4096 + 37


def _case(kind, rng, Q):
    """(fields, oracle aux, device aux, x [Q, n], level scale [Q], branch gap [Q] or None)."""
    if kind == "ball":
        n, dp = 3, (2, 0.8)
        x = rng.uniform(-2, 2, (Q, n))
        return dict(n=n, ham="quadratic", datum="ball", datum_p=dp, nu=0.05), None, None, x, None
    if kind == "disc_union":
        n, cen = 4, np.array([[1.2, 0.0], [-0.6, 1.0], [0.1, -1.3]], dtype=np.float32)
        x = rng.uniform(-2.5, 2.5, (Q, n))
        d = np.sort(np.hypot(x[:, None, 0] - cen[:, 0], x[:, None, 1] - cen[:, 1]), 1)
        return (dict(n=n, ham="quadratic", datum="disc_union", datum_p=(0.5, 3), nu=0.05), cen.astype(np.float64),
                to_dev(cen), x, d[:, 1] - d[:, 0])
    if kind == "half_sqnorm":
        n = 5
        x = rng.uniform(-1.5, 1.5, (Q, n))
        return dict(n=n, ham="quadratic", datum="half_sqnorm", nu=0.05), None, None, x, None
    if kind == "min_pair_disks":
        n = 9
        x = rng.uniform(-2, 2, (Q, n))
        r2 = np.sort(x[:, 0::3] ** 2 + x[:, 1::3] ** 2, 1)
        return (dict(n=n, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.6,), nu=0.01), None, None, x,
                np.sqrt(r2[:, 1]) - np.sqrt(r2[:, 0]))
    if kind == "capture":
        n = 48
        x = rng.uniform(-3, 3, (Q, n))
        dx, dy = x[:, 0:45:3] - x[:, 45:46], x[:, 1:45:3] - x[:, 46:47]
        d = np.sort(np.hypot(dx, dy), 1)
        return (dict(n=n, ham="pursuit_evasion", ham_p=(1.0, 1.0, 1.0), datum="capture", datum_p=(0.4,), nu=0.01),
                None, None, x, d[:, 1] - d[:, 0])
    if kind == "knn_balls":
        n, K = 6, 4
        x = rng.uniform(-2, 2, (Q, n))
        nb = rng.uniform(-2, 2, (Q, K, 3))
        d = np.sort(np.linalg.norm(x[:, None, :3] - nb, axis=-1), 1)
        dev = to_dev(np.ascontiguousarray(np.transpose(nb.astype(np.float32), (1, 2, 0))))   # [K][3][Q]
        return (dict(n=n, ham="double_integrator", ham_p=(1.0,), datum="knn_balls", datum_p=(0.3, K), nu=0.02),
                nb.astype(np.float32).astype(np.float64), dev, x, d[:, 1] - d[:, 0])
    if kind == "linear":
        n = 16
        a = rng.normal(size=n).astype(np.float32)
        x = rng.uniform(-1, 1, (Q, n))
        return (dict(n=n, ham="quadratic", datum="linear", datum_p=(0.3,), nu=0.05), a.astype(np.float64),
                to_dev(a), x, None)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["ball", "disc_union", "half_sqnorm", "min_pair_disks", "capture", "knn_balls",
                                  "linear"])
def test_projection_matches_oracle(ctx, kind):
    from paper_2605_18566_amd import avoid_project
    rng = np.random.default_rng(100 + len(kind))
    Q = Q_RAGGED
    fields, aux_or, aux_dev, x, gap = _case(kind, rng, Q)
    x = x.astype(np.float32).astype(np.float64)
    n = fields["n"]
    v = rng.uniform(-2.0, 2.0, Q).astype(np.float32)
    g = rng.normal(size=(Q, n)).astype(np.float32)
    print(f"[avoid] kind={kind} n={n} Q={Q}", flush=True)
    xd, vd, gd = to_dev(soa(x)), to_dev(v), to_dev(soa(g))
    act = avoid_project(gpu_problem(fields, aux=aux_dev), xd, vd, gd, want_active=True)
    torch.cuda.synchronize()
    vo, go, ao = vd.cpu().numpy(), gd.cpu().numpy().T, act.cpu().numpy().astype(bool)
    pb = oracle_problem(fields, aux=aux_or if kind != "knn_balls" else None)
    rv, rg, ra = avoid.project(pb, x, v.astype(np.float64), g.astype(np.float64),
                               aux_all=aux_or if kind == "knn_balls" else None)
    lv, _ = avoid.obstacle_level(pb, x, aux_or if kind == "knn_balls" else None)
    scale = np.abs(lv)
    if kind == "linear":
        scale = np.abs(x * aux_or).sum(1) + 0.3
    tol = 2e-6 * (1.0 + np.abs(lv) + scale)
    assert np.all(np.abs(vo - rv) <= tol), np.max(np.abs(vo - rv) - tol)
    clear = np.abs(-lv - v) > tol
    assert clear.mean() > 0.99 and ra.any() and (~ra).any()
    assert np.array_equal(ao[clear], ra[clear])
    kept = ~ao
    assert np.array_equal(vo[kept], v[kept]) and np.array_equal(go[kept], g[kept])
    on = ao & ra
    unique = on if gap is None else on & (gap > 1e-4)
    np.testing.assert_allclose(go[unique], rg[unique], rtol=0, atol=2e-6 * (1 + np.abs(rg[unique]).max()))
    other = on & ~unique
    if other.any() and kind != "linear" and kind != "half_sqnorm":
        # an equally near branch: still a unit-slope gradient of one branch
        nrm = np.linalg.norm(go[other], axis=1)
        assert np.all(np.abs(nrm - np.linalg.norm(rg[other], axis=1)) <= 1e-5)


def test_grad_optional_nan_kept_and_empty(ctx):
    from paper_2605_18566_amd import avoid_project
    rng = np.random.default_rng(7)
    fields, aux_or, aux_dev, x, _ = _case("disc_union", rng, 1000)
    spec = gpu_problem(fields, aux=aux_dev)
    v = rng.uniform(-2, 2, 1000).astype(np.float32)
    v[17] = np.nan
    g = rng.normal(size=(1000, 4)).astype(np.float32)
    xd = to_dev(soa(x))
    va, ga = to_dev(v), to_dev(soa(g))
    vb = to_dev(v)
    aa = avoid_project(spec, xd, va, ga, want_active=True)
    ab = avoid_project(spec, xd, vb, None, want_active=True)
    torch.cuda.synchronize()
    assert torch.equal(aa, ab)
    assert torch.equal(torch.nan_to_num(va, nan=123.0), torch.nan_to_num(vb, nan=123.0))
    assert np.isnan(va[17].item()) and aa[17].item() == 0
    # Q = 0 is a no-op; wrong shapes and an obstacle without its centres are errors
    e = torch.empty(4, 0, device="cuda")
    assert avoid_project(spec, e, torch.empty(0, device="cuda")) is None
    with pytest.raises(ValueError):
        avoid_project(spec, xd[:3].contiguous(), va)
    from paper_2605_18566_amd._lib import HJGError
    bad = gpu_problem(fields)                     # disc_union needs datum_aux
    with pytest.raises(HJGError):
        avoid_project(bad, xd, va)


@pytest.mark.parametrize("Q", [1, 2, 63, 65])
def test_one_dimension_and_tiny_batches(ctx, Q):
    """n = 1 (an interval as the avoid set) at batch sizes below and around one
    wave: values, flags and gradients equal the oracle's."""
    from paper_2605_18566_amd import avoid_project
    rng = np.random.default_rng(300 + Q)
    fields = dict(n=1, ham="quadratic", datum="ball", datum_p=(1, 0.5), nu=0.05)
    x = rng.uniform(-1.0, 1.0, (Q, 1)).astype(np.float32).astype(np.float64)
    v = rng.uniform(-1.0, 1.0, Q).astype(np.float32)
    g = rng.normal(size=(Q, 1)).astype(np.float32)
    vd, gd = to_dev(v), to_dev(soa(g))
    act = avoid_project(gpu_problem(fields), to_dev(soa(x)), vd, gd, want_active=True)
    torch.cuda.synchronize()
    rv, rg, ra = avoid.project(oracle_problem(fields), x, v.astype(np.float64), g.astype(np.float64))
    lv, _ = avoid.obstacle_level(oracle_problem(fields), x)
    tol = 2e-6 * (1.0 + np.abs(lv))
    clear = np.abs(-lv - v) > tol
    assert np.all(np.abs(vd.cpu().numpy() - rv) <= tol)
    a = act.cpu().numpy().astype(bool)
    assert np.array_equal(a[clear], ra[clear])
    np.testing.assert_allclose(gd.cpu().numpy().T[clear], rg[clear], rtol=0, atol=1e-6)


def test_reach_avoid_step_matches_oracle(ctx):
    """One reach-avoid time step on the relative Dubins tube (horizon 0.1,
    K = 3, tilt, common draws): Algorithm 1 then the projection onto a union
    of two discs in the relative plane, device against oracle."""
    from paper_2605_18566_amd import avoid_project, picard_sweep
    w = workloads.C2
    fields = dict(w.problem_fields())
    Q, N, K, t = 1200, 4096, 3, 0.1
    x = workloads.queries(w, Q=Q, trial=9).astype(np.float32).astype(np.float64)
    # one disc overlaps the capture disc (the projection carves the target),
    # one lies outside it
    cen = np.array([[0.6, 0.0], [-1.0, -1.2]], dtype=np.float32)
    obst = dict(n=3, ham="quadratic", datum="disc_union", datum_p=(0.45, 2), nu=0.05)
    print(f"[avoid] reach-avoid step Q={Q} N={N} K={K}", flush=True)
    out = picard_sweep(ctx, gpu_problem(fields), to_dev(soa(x)), t, N, K, time_step=1)
    act = avoid_project(gpu_problem(obst, aux=to_dev(cen)), to_dev(soa(x)), out.v, out.grad, want_active=True)
    torch.cuda.synchronize()
    pb = oracle_problem(fields)
    ref = estimator.picard(pb, x, t, N, K, time_step=1)
    rv, rg, ra = avoid.project(oracle_problem(obst, aux=cen.astype(np.float64)), x, ref.v, ref.grad)
    v = out.v.cpu().numpy()
    sigma = np.sqrt(pb.delta * t)
    vt = 10 * value_tol(ref.v, ref.c, ref.theta, sigma, ref.lmax) + 1e-5
    assert np.mean(np.abs(v - rv) <= vt) >= 0.995
    a = act.cpu().numpy().astype(bool)
    lv, _ = avoid.obstacle_level(oracle_problem(obst, aux=cen.astype(np.float64)), x)
    clear = np.abs(-lv - ref.v) > vt
    assert np.mean(a[clear] == ra[clear]) >= 0.995 and ra.sum() >= 10
    inside = lv < -1e-5
    assert inside.any() and np.all(v[inside] > 0)          # no state of the avoid set is reached
