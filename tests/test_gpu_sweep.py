"""Parity of the HIP sweep with the FP64 oracle (runs on an MI355X).

Both sides get the same seeded float32 inputs and draw the same Philox
streams; outputs are compared element by element at sizes that span several
blocks, several sample splits and ragged tails.
"""
import numpy as np
import pytest

import workloads
from oracle import estimator, model, philox
from tests._helpers import ESS_RTOL_CAP, ess_rtol, gpu_problem, grad_tol, oracle_problem, soa, to_dev, value_tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2605_18566_amd import Context
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    c = Context(0)
    yield c
    c.close()


# ------------------------------------------------------------------ draws
@pytest.mark.parametrize("seed,c1,c2,c3", [(0, 0, 0, 0), (0x0002605185660011, 3, 0xFFFFFFFF, 0x00010200),
                                           (2 ** 64 - 1, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)])
def test_philox_words_bit_exact(seed, c1, c2, c3):
    from paper_2605_18566_amd import philox_words
    G = 10000
    gpu = philox_words(seed, c1, c2, c3, G)
    k0, k1 = philox.split_seed(seed)
    ref = np.stack(philox.philox4x32_10(np.arange(G), c1, c2, c3, k0, k1), axis=1)
    np.testing.assert_array_equal(gpu, ref)


@pytest.mark.parametrize("n,N", [(3, 1000), (5, 4099), (1, 7)])
def test_table_normals_fp32_within_4ulp(ctx, n, N):
    from paper_2605_18566_amd import ProblemSpec, sample_table
    spec = ProblemSpec(n=n, datum="half_sqnorm", seed=0x1234567890ABCDEF, problem_id=7)
    z = sample_table(ctx, spec, N, time_step=3).cpu().numpy().astype(np.float64)
    ref = philox.crn_table(spec.seed, 7, 3, n, N)
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    err = np.abs(z - ref)
    assert np.all(err <= 4 * ulp + 1e-12), (err / ulp).max()


def test_table_normals_bf16(ctx):
    from paper_2605_18566_amd import ProblemSpec, sample_table
    n, N = 4, 50000
    spec = ProblemSpec(n=n, datum="half_sqnorm", seed=99, problem_id=1, sample_bf16=True)
    z = sample_table(ctx, spec, N, time_step=0).float().cpu().numpy().astype(np.float64)
    ref = philox.crn_table(99, 1, 0, n, N, bf16=True)
    mism = z != ref
    # double rounding (FP64 -> FP32 -> BF16 vs FP64 -> BF16) and FP32 ulps can
    # flip a value that sits on a bfloat16 rounding boundary: rare, one bf16 ulp
    assert mism.mean() <= 1e-3
    bf_ulp = np.spacing(np.abs(ref).astype(np.float32)) * 2 ** 16
    assert np.all(np.abs(z - ref)[mism] <= bf_ulp[mism] * 1.01)


# ---------------------------------------------------------- one frozen sweep
CASES = {
    # name: (workload fields, Q, N, tilt-from-datum-gradient)
    "quad_disk_fresh": (dict(workloads.C1.problem_fields()), 1000, 3001),
    "quad_disk_crn": (dict(workloads.C1.problem_fields(), sample_mode="crn_step"), 777, 5000),
    "quad_halfsq_crn_cv": (dict(workloads.C1_QUAD.problem_fields(), sample_mode="crn_step", grad_cv=True,
                                tilt=True), 513, 2048),
    "quad_halfsq_fresh_cv_bf16": (dict(workloads.C1_QUAD.problem_fields(), grad_cv=True, sample_bf16=True),
                                  300, 1027),
    "dubins_n3_tilt": (dict(workloads.C2.problem_fields()), 1500, 4096 + 77),
    "dubins_n3_printed_sign": (dict(workloads.C2.problem_fields(), ham_p=(-1.0, 1.0, 1.0, 1.0)), 600, 2000),
    "dubins_n3_plain_h": (dict(workloads.C2.problem_fields(), tube=False), 700, 3000),
    "dubins_n45_bf16": (dict(workloads.C5.problem_fields()), 600, 3000),
    "dubins_n12_fp32": (dict(workloads.C5.problem_fields(), n=12, sample_bf16=False), 700, 2500),
    "dubins_n30_bf16_cv": (dict(workloads.C5.problem_fields(), n=30, grad_cv=True), 400, 1500),
    "zero_ham_small_c": (dict(workloads.C2.problem_fields(), ham="zero", tilt=False, c_min=1e-3), 300, 2000),
    # matrix-core pair loop (bf16 common table, n >= 16); ragged Q and N
    "mfma_dubins_n45_ragged": (dict(workloads.C5.problem_fields()), 333, 1000 + 13),
    "mfma_dubins_n48_notilt": (dict(workloads.C5.problem_fields(), n=48, tilt=False), 260, 777),
    "mfma_dubins_n18_cv": (dict(workloads.C5.problem_fields(), n=18, grad_cv=True), 500, 2053),
    # bfloat16 common tables below n = 16 (vector-ALU loop)
    "dubins_n3_bf16": (dict(workloads.C2.problem_fields(), sample_bf16=True), 700, 3000 + 11),
    "dubins_n6_bf16_cv": (dict(workloads.C5.problem_fields(), n=6, grad_cv=True), 513, 1500),
    "dubins_n15_bf16_notilt": (dict(workloads.C5.problem_fields(), n=15, tilt=False), 400, 2048),
    "mfma_quad_halfsq_n20": (dict(workloads.C1_QUAD.problem_fields(), n=20, sample_mode="crn_step",
                                  sample_bf16=True, tilt=True), 300, 1500),
    "mfma_quad_ball_n16_k3": (dict(workloads.C1.problem_fields(), n=16, datum_p=(3, 1.0), sample_mode="crn_step",
                                   sample_bf16=True, tilt=True, grad_cv=True), 257, 999),
    # the multi-pursuer game: vector-ALU (n < 16, fp32, fresh) and matrix-core paths
    "pursuit_n9_fp32": (dict(workloads.C6.problem_fields(), n=9, sample_bf16=False, tilt=True), 700, 3001),
    "pursuit_n9_fresh": (dict(workloads.C6.problem_fields(), n=9, sample_mode="fresh", sample_bf16=False), 400, 2000),
    "pursuit_n45_fp32_valu": (dict(workloads.C6.problem_fields(), sample_bf16=False), 300, 1500),
    "mfma_pursuit_n45": (dict(workloads.C6.problem_fields(), tilt=True), 333, 2000 + 5),
    "mfma_pursuit_n18_slow_evader": (dict(workloads.C6.problem_fields(), n=18, ham_p=(1.0, 2.0, 1.0)), 400, 1800),
    # the two-rocket game (ball datum in (x, z)): fresh draws, and a common table with the shift
    "rockets_fresh": (dict(workloads.C7.problem_fields()), 700, 3001),
    "rockets_crn_tilt": (dict(workloads.C7.problem_fields(), sample_mode="crn_step", tilt=True), 500, 2048 + 3),
    # the paper's double integral plant (minimising control, disc about the origin)
    "dint_n2_fresh": (dict(workloads.C9.problem_fields()), 1000, 8000),
    "dint_n2_crn_tilt": (dict(workloads.C9.problem_fields(), sample_mode="crn_step", tilt=True), 700, 3001),
}


def _run_case(ctx, name, t=None):
    from paper_2605_18566_amd import value_grad
    fields, Q, N = CASES[name]
    n = fields["n"]
    w = workloads.C5 if n > 3 else (workloads.C2 if fields["ham"] != "quadratic" else workloads.C1)
    if fields["ham"] == "quadratic":
        w = workloads.C1
    if fields["ham"] == "rockets":
        box = ((-6.0, 6.0), (-6.0, 6.0), (-np.pi / 2, np.pi / 2))
    elif fields["datum"] == "min_pair_disks":
        box = workloads.dubins_box(n // 3)
    elif fields["datum"] == "capture":
        box = workloads.pursuit_box(n // 3, half=4.0)
    else:
        box = tuple([(-1.0, 1.0)] * n)
    x = workloads.queries(w.resized(n=n, box=box), Q=Q, trial=3).astype(np.float64)
    t = w.t if t is None else t
    pb = oracle_problem(fields)
    sigma = np.sqrt(pb.delta * t)
    p = model.datum_grad(pb, x)
    c = model.coefficient(pb, x, p).astype(np.float32).astype(np.float64)
    theta = model.tilt(pb, sigma, c, p).astype(np.float32).astype(np.float64)
    ref = estimator.value_grad(pb, x, t, N, c, theta if pb.tilt else None, time_step=2, iteration=1)
    spec = gpu_problem(fields)
    v, g, ess = value_grad(ctx, spec, to_dev(soa(x)), t, N, to_dev(c), to_dev(soa(theta)) if pb.tilt else None,
                           time_step=2, iteration=1, check_finite=True)
    torch.cuda.synchronize()
    return (v.cpu().numpy().astype(np.float64), g.cpu().numpy().T.astype(np.float64),
            ess.cpu().numpy().astype(np.float64), ref, c, theta if pb.tilt else None, sigma, N)


@pytest.mark.parametrize("name", list(CASES))
def test_value_grad_parity(ctx, name):
    v, g, ess, ref, c, theta, sigma, N = _run_case(ctx, name)
    print(f"[{name}] Q={len(v)} N={N}", flush=True)
    vt = value_tol(ref.v, c, theta if theta is not None else np.zeros_like(g), sigma, ref.lmax)
    dv = np.abs(v - ref.v)
    assert np.all(dv <= vt), f"value: worst {dv.max():.3e} (ratio {np.max(dv / vt):.2f})"
    gt = grad_tol(ref.grad, c, sigma, N)
    dg = np.linalg.norm(g - ref.grad, axis=1)
    assert np.all(dg <= gt), f"grad: worst ratio {np.max(dg / gt):.2f}"
    # ESS = S^2/S2 is not invariant to per-sample rounding of the log-weights
    # (|delta a| up to a few u32 |c| L each), unlike v's common-mode part.
    et = ess_rtol(c, theta, sigma, ref.lmax)
    rel = np.abs(ess - ref.ess) / ref.ess
    held = et <= ESS_RTOL_CAP
    print(f"[{name}] ESS rel err max {rel.max():.2e}, median {np.median(rel):.2e}; states held "
          f"{held.sum()} / {len(held)}", flush=True)
    assert np.all(rel[held] <= et[held]), f"ess: worst ratio {np.max(rel[held] / et[held]):.2f}"
    assert held.mean() >= 0.6          # 72 % for the shifted rocket game, all elsewhere


@pytest.mark.parametrize("name", ["mfma_dubins_n45_ragged", "mfma_quad_ball_n16_k3", "mfma_pursuit_n45"])
def test_valu_and_mfma_paths_agree(ctx, name, monkeypatch):
    a = _run_case(ctx, name)
    monkeypatch.setenv("HJG_NO_MFMA", "1")
    b = _run_case(ctx, name)
    ref, c, theta, sigma, N = a[3], a[4], a[5], a[6], a[7]
    th = theta if theta is not None else np.zeros_like(a[1])
    vt = value_tol(ref.v, c, th, sigma, ref.lmax)
    assert np.all(np.abs(a[0] - b[0]) <= 2 * vt)
    assert np.all(np.linalg.norm(a[1] - b[1], axis=1) <= 2 * grad_tol(ref.grad, c, sigma, N))


def test_value_grad_deterministic(ctx):
    a = _run_case(ctx, "dubins_n3_tilt")
    b = _run_case(ctx, "dubins_n3_tilt")
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_linear_datum_exact_on_gpu(ctx):
    # linear datum + Laplace shift: every log-weight is the same constant, so
    # the value is exact and ESS = N (tilted-proposal corollary)
    from paper_2605_18566_amd import value_grad
    a = np.array([0.6, -0.8, 0.3])
    fields = dict(n=3, ham="quadratic", datum="linear", nu=0.01, datum_p=(0.25,), tilt=True, grad_cv=True, seed=5)
    pb = oracle_problem(fields, aux=a)
    x = np.random.default_rng(0).uniform(-2, 2, (1000, 3)).astype(np.float32).astype(np.float64)
    t, N = 1.0, 4096
    sigma = np.sqrt(pb.delta * t)
    p = model.datum_grad(pb, x)
    c = model.coefficient(pb, x, p)
    theta = model.tilt(pb, sigma, c, p).astype(np.float32)
    spec = gpu_problem(fields, aux=to_dev(a))
    v, g, ess = value_grad(ctx, spec, to_dev(soa(x)), t, N, to_dev(c), to_dev(soa(theta)))
    v = v.cpu().numpy()
    np.testing.assert_allclose(v, x @ a + 0.25 - t * a @ a / 2, atol=2e-5)
    np.testing.assert_allclose(ess.cpu().numpy(), N, rtol=1e-5)
    np.testing.assert_allclose(g.cpu().numpy().T, np.tile(a, (1000, 1)), atol=2e-4)


def test_knn_datum_parity(ctx):
    from paper_2605_18566_amd import value_grad
    rng = np.random.default_rng(11)
    Q, K, N, t = 700, 7, 3000, 1.0
    x = np.concatenate([rng.uniform(0, 5, (Q, 3)), rng.normal(0, 0.5, (Q, 3))], 1).astype(np.float32).astype(np.float64)
    nb = (x[:, None, :3] + rng.normal(0, 0.4, (Q, K, 3))).astype(np.float32).astype(np.float64)
    fields = dict(n=6, ham="double_integrator", ham_p=(1.0,), datum="knn_balls", datum_p=(0.2, K), nu=0.02,
                  tilt=True, seed=77)
    pb = oracle_problem(fields, aux=nb)
    sigma = np.sqrt(pb.delta * t)
    p = model.datum_grad(pb, x, nb)
    c = model.coefficient(pb, x, p).astype(np.float32).astype(np.float64)
    theta = model.tilt(pb, sigma, c, p).astype(np.float32).astype(np.float64)
    ref = estimator.value_grad(pb, x, t, N, c, theta)
    aux = to_dev(np.ascontiguousarray(np.transpose(nb, (1, 2, 0))))       # [K][3][Q]
    spec = gpu_problem(fields, aux=aux)
    v, g, ess = value_grad(ctx, spec, to_dev(soa(x)), t, N, to_dev(c), to_dev(soa(theta)))
    v, g = v.cpu().numpy(), g.cpu().numpy().T
    assert np.all(np.abs(v - ref.v) <= value_tol(ref.v, c, theta, sigma, ref.lmax))
    assert np.all(np.linalg.norm(g - ref.grad, axis=1) <= grad_tol(ref.grad, c, sigma, N))


# ------------------------------------------------------------ Picard loop
def _picard_both(ctx, fields, Q, N, K, t, tol=0.0, trial=4, w=workloads.C2, box=None, graph=True):
    from paper_2605_18566_amd import picard_sweep
    box = box or w.box
    x = workloads.queries(w.resized(n=fields["n"], box=box), Q=Q, trial=trial).astype(np.float64)
    pb = oracle_problem(fields)
    ref = estimator.picard(pb, x, t, N, K, tol=tol, time_step=1)
    out = picard_sweep(ctx, gpu_problem(fields), to_dev(soa(x)), t, N, K, tol=tol, time_step=1)
    torch.cuda.synchronize()
    return out, ref, pb


def test_picard_c1_single_iteration(ctx):
    fields = dict(workloads.C1.problem_fields())
    out, ref, pb = _picard_both(ctx, fields, 2000, 4000, 1, 0.5, w=workloads.C1)
    v = out.v.cpu().numpy()
    sigma = np.sqrt(pb.delta * 0.5)
    assert np.all(np.abs(v - ref.v) <= value_tol(ref.v, ref.c, np.zeros((2000, 2)), sigma, ref.lmax))
    g = out.grad.cpu().numpy().T
    assert np.all(np.linalg.norm(g - ref.grad, axis=1) <= grad_tol(ref.grad, ref.c, sigma, 4000))
    assert out.iters_done == 1
    np.testing.assert_allclose(out.resid_hist, ref.resid_hist, rtol=1e-4)


def test_picard_dubins_multi_iteration(ctx):
    # K = 3 with the tilt from the previous iterate: float32 differences in the
    # iterate feed the next coefficient, so compare with a per-query tolerance
    # scaled by the iteration count and require almost every query inside it.
    fields = dict(workloads.C2.problem_fields())
    assert fields["tube"]
    Q, N, K, t = 1200, 4096, 3, 1.0
    out, ref, pb = _picard_both(ctx, fields, Q, N, K, t)
    sigma = np.sqrt(pb.delta * t)
    v = out.v.cpu().numpy()
    vt = 10 * value_tol(ref.v, ref.c, ref.theta, sigma, ref.lmax)
    frac = np.mean(np.abs(v - ref.v) <= vt)
    print(f"[picard dubins] within tol: {frac:.4f}, max |dv| {np.abs(v - ref.v).max():.2e}")
    assert frac >= 0.995
    np.testing.assert_allclose(out.resid_hist, ref.resid_hist, rtol=2e-2, atol=1e-6)
    c = out.c.cpu().numpy()
    assert np.mean(np.abs(c - ref.c) <= 1e-3 * np.abs(ref.c) + 1e-3) >= 0.99
    assert np.all(ref.c <= pb.c_min)             # min{0, H}: never a positive coefficient above c_min


def test_picard_pursuit_game(ctx):
    # the 45-dimensional multi-pursuer game (tube coefficient, tilt, bf16 draws)
    w = workloads.C6
    fields = dict(w.problem_fields())
    Q, N, K, t = 300, 4096, 5, 1.0
    out, ref, pb = _picard_both(ctx, fields, Q, N, K, t, trial=8, w=w, box=workloads.pursuit_box(15, half=4.0))
    sigma = np.sqrt(pb.delta * t)
    v = out.v.cpu().numpy()
    vt = 10 * value_tol(ref.v, ref.c, ref.theta, sigma, ref.lmax)
    dv = np.abs(v - ref.v)
    bad = dv > vt
    # float32 rounding of one iterate moves the next iteration's shift theta,
    # i.e. its proposal; where |c| is large and the ESS small the estimate then
    # moves within its Monte-Carlo band: SE(v) ~ sqrt((N/ESS - 1)/N)/|c|
    se = np.sqrt(np.maximum(N / ref.ess - 1.0, 0.0) / N) / np.abs(ref.c)
    c = out.c.cpu().numpy()
    print(f"[picard pursuit] within tol: {1 - bad.mean():.4f}, max |dv| {dv.max():.2e}; outside: |c| "
          f"{np.abs(c[bad]).round(2).tolist()}, ESS {ref.ess[bad].round(1).tolist()}, |dv|/SE "
          f"{(dv[bad] / se[bad]).round(2).tolist()}", flush=True)
    assert bad.mean() <= 0.02
    assert np.all(dv[bad] <= 3 * se[bad])
    np.testing.assert_allclose(out.resid_hist, ref.resid_hist, rtol=5e-2, atol=1e-6)


@pytest.mark.parametrize("tilt", [False, True], ids=["plain", "tilt"])
def test_picard_double_integral_plant(ctx, tilt):
    # the paper's double integral plant at its table's setting (N = 8,000 fresh
    # draws, delta = 0.08, K = 15) on a 32 x 32 grid, horizon 0.8.  With the
    # Laplace shift the proposal follows the gradient iterate, so a float32
    # difference moves later proposals as well: that chain is compared over
    # K = 5 (as the other shifted multi-iteration checks)
    fields = dict(workloads.C9.problem_fields(), tilt=tilt)
    Q, N, K, t = 1024, 8000, (5 if tilt else 15), 0.8
    x = workloads.dint_grid(32).astype(np.float64)
    pb = oracle_problem(fields)
    from paper_2605_18566_amd import picard_sweep
    ref = estimator.picard(pb, x, t, N, K, time_step=1)
    out = picard_sweep(ctx, gpu_problem(fields), to_dev(soa(x)), t, N, K, time_step=1)
    torch.cuda.synchronize()
    sigma = np.sqrt(pb.delta * t)
    v = out.v.cpu().numpy()
    vt = 10 * value_tol(ref.v, ref.c, ref.theta, sigma, ref.lmax)
    # fifteen iterations on fresh draws: a float32 difference in one iterate
    # moves every later coefficient, and each iteration's estimate moves
    # within its own band, so the band is 4 standard errors over 15
    # iterations (3 over five)
    se = (4 if K > 5 else 3) * np.sqrt(np.maximum(N / ref.ess - 1.0, 0.0) / N) / np.abs(ref.c)
    dv = np.abs(v - ref.v)
    print(f"[double integrator, tilt={tilt}] within 10 tol {np.mean(dv <= vt):.4f}, max |dv| {dv.max():.2e}, "
          f"residuals {np.round(out.resid_hist[-3:], 4).tolist()} (oracle {np.round(ref.resid_hist[-3:], 4).tolist()})",
          flush=True)
    assert np.all(dv <= np.maximum(vt, se))
    assert np.mean(dv <= vt) >= 0.98
    np.testing.assert_allclose(out.resid_hist, ref.resid_hist, rtol=5e-2, atol=1e-6)
    assert out.iters_done == K


def test_picard_dubins_plain_h(ctx):
    fields = dict(workloads.C2.problem_fields(), tube=False)
    Q, N, K, t = 1000, 4096, 3, 1.0
    out, ref, pb = _picard_both(ctx, fields, Q, N, K, t, trial=6)
    sigma = np.sqrt(pb.delta * t)
    v = out.v.cpu().numpy()
    vt = 10 * value_tol(ref.v, ref.c, ref.theta, sigma, ref.lmax)
    assert np.mean(np.abs(v - ref.v) <= vt) >= 0.995


def test_picard_early_exit(ctx):
    fields = dict(workloads.C1.problem_fields(), sample_mode="crn_step")
    out, ref, pb = _picard_both(ctx, fields, 1000, 2048, 6, 0.5, tol=1e-6, w=workloads.C1)
    assert ref.iters_done == 2
    assert out.iters_done == 2
    assert out.status == 0
    assert out.resid_hist[1] == 0.0 and np.all(out.resid_hist[2:] == 0.0)


def test_picard_graph_replay_matches_direct(ctx, monkeypatch):
    from paper_2605_18566_amd import picard_sweep
    fields = dict(workloads.C2.problem_fields())
    x = to_dev(soa(workloads.queries(workloads.C2, Q=900, trial=9)))
    spec = gpu_problem(fields)
    outs = []
    for _ in range(3):                     # first call records, later calls replay
        o = picard_sweep(ctx, spec, x, 1.0, 2048, 3)
        outs.append((o.v.clone(), o.grad.clone(), o.resid_hist.copy()))
        torch.cuda.synchronize()
    monkeypatch.setenv("HJG_NO_GRAPH", "1")
    d = picard_sweep(ctx, spec, x, 1.0, 2048, 3)
    for v, g, h in outs:
        assert torch.equal(v, d.v) and torch.equal(g, d.grad)
        np.testing.assert_array_equal(h, d.resid_hist)


# ------------------------------------------------------------------ edges
def test_empty_and_invalid(ctx):
    from paper_2605_18566_amd import picard_sweep, value_grad
    from paper_2605_18566_amd._lib import HJGError
    spec = gpu_problem(dict(workloads.C1.problem_fields()))
    x0 = torch.empty((2, 0), device="cuda")
    v, g, e = value_grad(ctx, spec, x0, 0.5, 100, torch.empty(0, device="cuda"))
    assert v.numel() == 0
    out = picard_sweep(ctx, spec, x0, 0.5, 100, 2)
    assert out.iters_done == 0
    x = to_dev(np.zeros((2, 4)))
    c = to_dev(np.ones(4))
    with pytest.raises(HJGError):
        value_grad(ctx, spec, x, -1.0, 100, c)         # t <= 0
    with pytest.raises(HJGError):
        value_grad(ctx, spec, x, 0.5, 0, c)            # N = 0
    bad = gpu_problem(dict(workloads.C1.problem_fields(), nu=0.0))
    with pytest.raises(HJGError):
        value_grad(ctx, bad, x, 0.5, 100, c)
    wide = gpu_problem(dict(workloads.C5.problem_fields(), sample_mode="fresh"))
    with pytest.raises(HJGError):
        value_grad(ctx, wide, to_dev(np.zeros((45, 4))), 1.0, 100, c)


def test_single_sample_and_single_query(ctx):
    from paper_2605_18566_amd import value_grad
    fields = dict(workloads.C2.problem_fields(), tilt=False)
    pb = oracle_problem(fields)
    x = np.array([[0.7, -0.4, 0.3]])
    c = np.array([3.0])
    for N in (1, 2, 5):
        ref = estimator.value_grad(pb, x, 1.0, N, c)
        v, g, e = value_grad(ctx, gpu_problem(fields), to_dev(soa(x)), 1.0, N, to_dev(c))
        np.testing.assert_allclose(v.cpu().numpy(), ref.v, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(e.cpu().numpy(), ref.ess, rtol=1e-5)


def test_timing_hook_keeps_results(ctx):
    from paper_2605_18566_amd import picard_sweep
    fields = dict(workloads.C2.problem_fields())
    x = to_dev(soa(workloads.queries(workloads.C2, Q=800, trial=12)))
    spec = gpu_problem(fields)
    a = picard_sweep(ctx, spec, x, 1.0, 2048, 4)
    ctx.set_timing(True)
    try:
        b = picard_sweep(ctx, spec, x, 1.0, 2048, 4)
        ms, launches = ctx.sweep_time()
        b2 = picard_sweep(ctx, spec, x, 1.0, 2048, 4)     # replay of the timed graph
        ms2, launches2 = ctx.sweep_time()
    finally:
        ctx.set_timing(False)
    assert launches == 4 and launches2 == 4 and ms > 0 and ms2 > 0
    assert torch.equal(a.v, b.v) and torch.equal(a.grad, b.grad) and torch.equal(b.v, b2.v)
