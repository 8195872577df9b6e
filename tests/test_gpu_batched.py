"""Many uneven problems in one batched call vs one call per problem and vs the
FP64 oracle (runs on an MI355X)."""
import numpy as np
import pytest

import workloads
from oracle import estimator
from tests._helpers import gpu_problem, oracle_problem, soa, to_dev, value_tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2605_18566_amd import Context
    c = Context(0)
    yield c
    c.close()


def small_batch(P=14, scale=0.03, trial=1):
    batch = workloads.c3_batch(P=P, scale=scale, trial=trial)
    xs = [np.ascontiguousarray(workloads.queries(bp.w, trial=7 + i).T) for i, bp in enumerate(batch)]
    return batch, xs


def run_batched(ctx, batch, xs, tol=0.0):
    from paper_2605_18566_amd import picard_sweep_batched
    specs = [gpu_problem(workloads.c3_fields(bp), problem_id=bp.problem_id) for bp in batch]
    return picard_sweep_batched(ctx, specs, [to_dev(x) for x in xs], [bp.w.N for bp in batch],
                                [bp.w.K for bp in batch], [bp.w.t for bp in batch], tol=tol)


def split_out(out, batch):
    vs, gs = [], []
    for p, bp in enumerate(batch):
        vs.append(out.v[out.q_off[p]:out.q_off[p + 1]].cpu().numpy())
        gs.append(out.grad[out.x_off[p]:out.x_off[p + 1]].reshape(bp.w.n, -1).cpu().numpy())
    return vs, gs


def test_batch_spans_both_pair_loops_and_uneven_k():
    batch, _ = small_batch()
    ns = [bp.w.n for bp in batch]
    assert min(ns) < 16 <= max(ns)
    assert len({bp.w.K for bp in batch}) > 1


def test_batched_is_bit_identical_to_one_call_per_problem(ctx, monkeypatch):
    # one sample split per problem on both paths: the same arithmetic in the
    # same order, so every iterate must agree bit for bit
    from paper_2605_18566_amd import picard_sweep
    monkeypatch.setenv("HJG_TARGET_BLOCKS", "1")
    monkeypatch.setenv("HJG_BATCH_SPLIT", str(1 << 30))
    batch, xs = small_batch()
    out = run_batched(ctx, batch, xs)
    vs, gs = split_out(out, batch)
    for p, bp in enumerate(batch):
        spec = gpu_problem(workloads.c3_fields(bp), problem_id=bp.problem_id)
        one = picard_sweep(ctx, spec, to_dev(xs[p]), bp.w.t, bp.w.N, bp.w.K)
        print(f"[problem {p}] n={bp.w.n} Q={bp.w.Q} N={bp.w.N} K={bp.w.K} nu={bp.w.nu:.3g}", flush=True)
        assert out.iters[p] == one.iters_done == bp.w.K
        np.testing.assert_array_equal(vs[p], one.v.cpu().numpy())
        np.testing.assert_array_equal(gs[p], one.grad.cpu().numpy())
        np.testing.assert_array_equal(out.resid_hist[p, :bp.w.K], one.resid_hist)


def test_batched_first_iteration_matches_with_default_splits(ctx):
    # default plans cut the samples differently (float64 merge order differs);
    # with K = 1 nothing feeds back, so every state agrees to rounding
    from paper_2605_18566_amd import picard_sweep
    batch, xs = small_batch()
    for bp in batch:
        bp.w = bp.w.resized(K=1)
    out = run_batched(ctx, batch, xs)
    vs, _ = split_out(out, batch)
    for p, bp in enumerate(batch):
        spec = gpu_problem(workloads.c3_fields(bp), problem_id=bp.problem_id)
        one = picard_sweep(ctx, spec, to_dev(xs[p]), bp.w.t, bp.w.N, 1)
        v1, c1 = one.v.cpu().numpy(), one.c.cpu().numpy().astype(np.float64)
        # the float32 rounding terms of the value tolerance (tests/_helpers.py):
        # S differs at ~128 u32 relative between split plans, and v = -(1/c) ln S
        # scales that by 1/|c| (|c| = c_min = 0.01 where min{0, H} = 0)
        U32 = 2.0 ** -24
        tol = 1e-4 * np.abs(v1) + 64 * U32 * 10 + 128 * U32 / np.abs(c1)
        assert np.all(np.abs(vs[p] - v1) <= tol), np.max(np.abs(vs[p] - v1) / tol)


def test_batched_first_iteration_matches_oracle(ctx):
    # the batched path is bit-identical to the single-problem path (above),
    # which the Picard parity tests cover over several iterations; here every
    # problem of the batch is checked against the oracle where nothing feeds
    # back (K = 1): every state within the value tolerance
    batch, xs = small_batch()
    for bp in batch:
        bp.w = bp.w.resized(K=1)
    out = run_batched(ctx, batch, xs)
    vs, _ = split_out(out, batch)
    picked = [p for p, bp in enumerate(batch) if bp.w.Q * bp.w.N <= 3_000_000]
    assert len(picked) >= 3
    for p in picked:
        bp = batch[p]
        pb = oracle_problem(workloads.c3_fields(bp))
        pb.problem_id = bp.problem_id
        ref = estimator.picard(pb, xs[p].T.astype(np.float64), bp.w.t, bp.w.N, 1)
        sigma = np.sqrt(pb.delta * bp.w.t)
        vt = value_tol(ref.v, ref.c, ref.theta, sigma, ref.lmax)
        print(f"[oracle {p}] n={bp.w.n} Q={bp.w.Q} N={bp.w.N} worst ratio {np.max(np.abs(vs[p] - ref.v) / vt):.3f}",
              flush=True)
        assert np.all(np.abs(vs[p] - ref.v) <= vt)


def test_batched_replay_is_deterministic(ctx):
    batch, xs = small_batch(P=8, trial=2)
    a = run_batched(ctx, batch, xs)
    va, ga = a.v.clone(), a.grad.clone()
    b = run_batched(ctx, batch, xs)     # same arguments: replays the recorded graph
    assert torch.equal(va, b.v) and torch.equal(ga, b.grad)
    np.testing.assert_array_equal(a.resid_hist, b.resid_hist)


def test_batched_stops_each_problem_on_its_own(ctx):
    from paper_2605_18566_amd import picard_sweep
    batch, xs = small_batch(P=8, trial=3)
    tol = 0.05
    out = run_batched(ctx, batch, xs, tol=tol)
    for p, bp in enumerate(batch):
        spec = gpu_problem(workloads.c3_fields(bp), problem_id=bp.problem_id)
        one = picard_sweep(ctx, spec, to_dev(xs[p]), bp.w.t, bp.w.N, bp.w.K, tol=tol)
        assert out.iters[p] == one.iters_done
        assert np.all(out.resid_hist[p, out.iters[p]:] == 0.0)


def test_persistent_launch_matches_one_block_per_item(monkeypatch):
    # the work queue only changes which block serves an item, so results are
    # bit-identical to the launch with one block per item
    from paper_2605_18566_amd import Context
    batch, xs = small_batch(P=10, trial=5)
    outs = []
    for mode in ("1", "0"):
        monkeypatch.setenv("HJG_BATCH_PERSISTENT", mode)
        c = Context(0)
        o = run_batched(c, batch, xs)
        outs.append((o.v.clone(), o.grad.clone(), o.resid_hist.copy()))
        c.close()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    np.testing.assert_array_equal(outs[0][2], outs[1][2])


def test_parallel_chains_match_one_chain(monkeypatch):
    # the specialisation chains as parallel graph branches or recorded one
    # after another: the same launches in another order, so the same bits
    from paper_2605_18566_amd import Context
    batch, xs = small_batch(P=12, trial=6)
    assert len({(bp.w.n, bp.w.n >= 16) for bp in batch}) > 2
    outs = []
    for mode in ("1", "0"):
        monkeypatch.setenv("HJG_BATCH_CONCURRENT", mode)
        c = Context(0)
        o = run_batched(c, batch, xs)
        outs.append((o.v.clone(), o.grad.clone(), o.resid_hist.copy(), o.iters.copy()))
        c.close()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    np.testing.assert_array_equal(outs[0][2], outs[1][2])
    np.testing.assert_array_equal(outs[0][3], outs[1][3])
