"""hjg_value_grad_noalloc against hjg_value_grad (runs on an MI355X).

The no-allocation entry point runs the same plan and kernels with its scratch
in the library's fixed per-GPU array, so its outputs must equal those of the
allocating entry point bit for bit.  Two calls in a row, the second with a
smaller input, check that nothing of the first call's scratch leaks into the
second.
"""
import numpy as np
import pytest

import workloads
from oracle import model
from tests._helpers import gpu_problem, oracle_problem, soa, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2605_18566_amd import Context
    c = Context(0)
    yield c
    c.close()


CASES = {
    # name: (fields, box workload, [(Q, N), (Q, N)] for the two calls)
    "crn_bf16_pairs_n45": (dict(workloads.C5.problem_fields()), workloads.C5, [(70000, 5000), (1333, 777)]),
    "crn_fp32_n3_cv": (dict(workloads.C2.problem_fields(), grad_cv=True), workloads.C2, [(20000, 4099), (513, 300)]),
    "fresh_n2_cv": (dict(workloads.C1.problem_fields(), grad_cv=True), workloads.C1, [(9000, 3001), (64, 129)]),
}


def _inputs(fields, w, Q, trial):
    x = workloads.queries(w.resized(n=fields["n"]), Q=Q, trial=trial).astype(np.float64)
    pb = oracle_problem(fields)
    sigma = np.sqrt(pb.delta * w.t)
    p = model.datum_grad(pb, x)
    c = model.coefficient(pb, x, p).astype(np.float32)
    theta = model.tilt(pb, sigma, c.astype(np.float64), p).astype(np.float32) if pb.tilt else None
    return to_dev(soa(x)), to_dev(c), (to_dev(soa(theta)) if theta is not None else None)


@pytest.mark.parametrize("name", list(CASES))
def test_noalloc_equals_value_grad_on_two_calls(ctx, name):
    from paper_2605_18566_amd import value_grad, value_grad_noalloc
    fields, w, sizes = CASES[name]
    spec = gpu_problem(fields)
    for call, (Q, N) in enumerate(sizes):
        print(f"[{name}] call {call}: Q={Q} N={N}", flush=True)
        x, c, theta = _inputs(fields, w, Q, 10 + call)
        a = value_grad_noalloc(ctx, spec, x, w.t, N, c, theta, time_step=1, iteration=2)
        b = value_grad(ctx, spec, x, w.t, N, c, theta, time_step=1, iteration=2)
        torch.cuda.synchronize()
        for got, ref in zip(a, b):
            np.testing.assert_array_equal(got.cpu().numpy(), ref.cpu().numpy())
        assert np.all(np.isfinite(a[0].cpu().numpy()))


def test_noalloc_rejects_inputs_beyond_its_scratch(ctx):
    from paper_2605_18566_amd import value_grad_noalloc
    from paper_2605_18566_amd._lib import HJG_EINVAL, HJGError
    fields = dict(workloads.C5.problem_fields())
    spec = gpu_problem(fields)
    Q = 1 << 20                       # 1M states x (20 + 180) bytes of partials > 128 MiB
    x = torch.zeros((45, Q), device="cuda")
    c = torch.ones(Q, device="cuda")
    with pytest.raises(HJGError) as ei:
        value_grad_noalloc(ctx, spec, x, 1.0, 4096, c)
    assert ei.value.code == HJG_EINVAL and "bytes of scratch" in str(ei.value)
