"""Certification kernels against the oracle (runs on an MI355X): labels and
population counts bit-exact (the comparison is made in float64 on both
sides, ties at the margin included), sampling margins to float32 rounding
with the same infinite entries, and the margin of a device sweep."""
import numpy as np
import pytest

from oracle import certify as oc
from oracle import estimator, model
from tests._helpers import gpu_problem, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("Q,with_margin", [(1, False), (1000, True), (300001, True), (4096, False)])
def test_labels_and_counts_bit_exact(Q, with_margin):
    from paper_2605_18566_amd import certify
    rng = np.random.default_rng(Q)
    v = rng.normal(0, 0.5, Q).astype(np.float32)
    E = 0.25
    m = rng.uniform(0, 0.2, Q).astype(np.float32) if with_margin else None
    v[: Q // 7] = np.float32(E)                        # ties at the margin: undetermined
    if m is not None:
        v[Q // 7: Q // 5] = -(np.float32(E) + m[Q // 7: Q // 5])
    lab, cnt = certify(to_dev(v), E, None if m is None else to_dev(m))
    ref = oc.classify(v, E, m)
    np.testing.assert_array_equal(lab.cpu().numpy(), ref)
    np.testing.assert_array_equal(cnt.cpu().numpy(), [np.sum(ref == -1), np.sum(ref == 0), np.sum(ref == 1)])


def test_empty_population_counts_zero():
    from paper_2605_18566_amd import _lib
    cnt = torch.full((3,), 7, dtype=torch.int64, device="cuda")
    assert _lib.lib().hjg_certify(0, None, None, 0.1, None, cnt.data_ptr(), None) == 0
    assert cnt.cpu().tolist() == [0, 0, 0]


def test_margins_match_oracle():
    from paper_2605_18566_amd import mc_margin
    rng = np.random.default_rng(5)
    Q = 50000
    v = rng.normal(0, 1, Q).astype(np.float32)
    c = (rng.choice([-1, 1], Q) * np.exp(rng.uniform(np.log(1e-2), np.log(50), Q))).astype(np.float32)
    ess = rng.uniform(1.0, 8192.0, Q).astype(np.float32)
    for g_min, g_max, bern in ((-0.5, np.inf, False), (-0.5, 4.0, False), (0.0, 1.0, False), (-0.5, np.inf, True),
                               (0.0, 1.0, True)):
        got = mc_margin(to_dev(v), to_dev(c), 8192, 0.05, g_min, g_max,
                        ess=to_dev(ess) if bern else None).cpu().numpy()
        ref = (oc.bernstein_margin(v, c, ess, 8192, 0.05, g_min, g_max) if bern
               else oc.mc_margin(v, c, 8192, 0.05, g_min, g_max))
        fin = np.isfinite(ref)
        np.testing.assert_array_equal(np.isfinite(got), fin)
        # float32 output: margins below its normal range flush to zero
        np.testing.assert_allclose(got[fin], ref[fin], rtol=2e-6, atol=1.2e-38)
        print(f"[margin g in [{g_min}, {g_max}] bernstein={bern}] finite {fin.mean():.3f}, "
              f"median {np.median(ref[fin]):.3e}", flush=True)


def test_margin_of_a_device_sweep_covers_the_exact_value():
    # plain estimator, exact quadratic case: the device value is within the
    # device margin of the closed form at every state (confidence 0.9)
    from paper_2605_18566_amd import Context, certify, mc_margin, value_grad
    ctx = Context(0)
    nu, t, N = 0.25, 0.5, 4096
    fields = dict(n=2, ham="quadratic", datum="half_sqnorm", nu=nu, sample_mode="fresh", seed=3)
    x = np.random.default_rng(1).uniform(-1, 1, (5000, 2))
    c = np.full(5000, 1.0 / (2 * nu), dtype=np.float32)
    v, _, ess = value_grad(ctx, gpu_problem(fields), to_dev(np.ascontiguousarray(x.T)), t, N, to_dev(c))
    exact = np.sum(x * x, 1) / (2 * (1 + t)) + 2 * nu * np.log1p(t)
    err = np.abs(v.cpu().numpy() - exact)
    mh = mc_margin(v, to_dev(c), N, 0.1, 0.0)
    assert np.all(err < mh.cpu().numpy())
    m = mc_margin(v, to_dev(c), N, 0.1, 0.0, ess=ess)
    assert np.mean(err < m.cpu().numpy()) >= 0.9
    # certify the sign of v - 0.5 (the sub-level set v <= 0.5) with the margin
    lab, cnt = certify(v - 0.5, 0.0, m)
    truth = exact - 0.5
    labs = lab.cpu().numpy()
    assert not np.any((labs == 1) & (truth <= 0)) and not np.any((labs == -1) & (truth > 0))
    print(f"[sweep certification] counts {cnt.cpu().tolist()}", flush=True)
    ctx.close()
