"""The autotuner: it picks one of its candidates, what it picks changes only the
summation order (results stay within the parity tolerance), and its table
survives a save/load round trip (runs on an MI355X)."""
import numpy as np
import pytest

import workloads
from oracle import estimator
from tests._helpers import gpu_problem, oracle_problem, to_dev, value_tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2605_18566_amd import Context
    c = Context(0)
    yield c
    c.close()


def test_autotune_sweep_keeps_parity(ctx, tmp_path):
    from paper_2605_18566_amd import Context, autotune_sweep, value_grad
    w = workloads.C5.resized(Q=512, N=4096)
    pb = oracle_problem(w.problem_fields())
    x = workloads.queries(w, trial=3).astype(np.float64)
    sigma = np.sqrt(pb.delta * w.t)
    c = np.full(w.Q, 0.7, dtype=np.float32).astype(np.float64)
    theta = (-0.3 * sigma * np.ones((w.Q, w.n))).astype(np.float32).astype(np.float64)
    ref = estimator.value_grad(pb, x, w.t, w.N, c, theta, 0, 0)
    spec = gpu_problem(w.problem_fields())
    xd, cd = to_dev(x.T.astype(np.float32)), to_dev(c.astype(np.float32))
    td = to_dev(theta.T.astype(np.float32))
    blocks, ms = autotune_sweep(ctx, spec, xd, w.t, w.N, cd, td)
    print(f"[autotune sweep] blocks={blocks} ms={ms:.4f}", flush=True)
    assert blocks in (512, 1024, 2048, 4096, 8192, 16384) and ms > 0
    v, g, _ = value_grad(ctx, spec, xd, w.t, w.N, cd, td)
    vt = value_tol(ref.v, c, theta, sigma, ref.lmax)
    assert np.all(np.abs(v.cpu().numpy() - ref.v) <= vt)
    path = tmp_path / "tuning.txt"
    ctx.save_tuning(path)
    text = path.read_text()
    assert text.startswith("hjg-tuning gfx950 1\n") and f"= {blocks}" in text
    other = Context(0)
    other.load_tuning(path)
    other.save_tuning(tmp_path / "again.txt")
    assert (tmp_path / "again.txt").read_text() == text
    (tmp_path / "bad.txt").write_text("something else\n")
    with pytest.raises(RuntimeError):
        other.load_tuning(tmp_path / "bad.txt")
    other.close()


def test_autotune_batched_choice_is_the_plan_it_runs(ctx, monkeypatch, tmp_path):
    # after tuning, the default batched call must be bit-identical to one that
    # forces the chosen samples-per-split, and to one in the other launch mode
    # (one block per item, one chain); the chosen mode is in the saved table
    from paper_2605_18566_amd import autotune_batched, picard_sweep_batched
    batch = workloads.c3_batch(P=10, scale=0.03, trial=4)
    xs = [to_dev(np.ascontiguousarray(workloads.queries(bp.w, trial=11 + i).T)) for i, bp in enumerate(batch)]
    specs = [gpu_problem(workloads.c3_fields(bp), problem_id=bp.problem_id) for bp in batch]
    args = ([bp.w.N for bp in batch], [bp.w.K for bp in batch], [bp.w.t for bp in batch])
    split, ms = autotune_batched(ctx, specs, xs, *args)
    print(f"[autotune batched] split={split} ms={ms:.3f}", flush=True)
    assert split in (2048, 4096, 8192, 16384, 32768, 65536) and ms > 0
    a = picard_sweep_batched(ctx, specs, xs, *args)
    va = a.v.clone()
    monkeypatch.setenv("HJG_BATCH_SPLIT", str(split))
    b = picard_sweep_batched(ctx, specs, xs, *args)
    assert torch.equal(va, b.v)
    path = str(tmp_path / "tuning.txt")
    ctx.save_tuning(path)
    entries = dict(line.split(" = ") for line in open(path).read().splitlines()[1:])
    assert int(entries["batch"]) == split and 1 <= int(entries["batch_mode"]) <= 4
    monkeypatch.setenv("HJG_BATCH_PERSISTENT", "0")
    monkeypatch.setenv("HJG_BATCH_CONCURRENT", "0")
    c = picard_sweep_batched(ctx, specs, xs, *args)
    assert torch.equal(va, c.v)
