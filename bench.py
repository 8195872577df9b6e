"""Throughput of the Monte-Carlo Picard sweep on one MI355X.

One step = one full Picard sweep (Algorithm 1: K frozen-coefficient
iterations, each drawing N samples per query and returning v and Dv) over the
n = 45 workload: 15 stacked relative Dubins pairs (tube coefficient
min{0, H}), 262,144 queries, N = 65,536 bfloat16 common draws, K = 5,
nu = 0.01, t = 1, Laplace shift from the previous iterate.  The metric is query.samples per second:
Q * N * K / (seconds per step).

Prints one JSON line with the throughput, the roofline of the dominant kernel
(the pair loop, timed by HIP events around every launch inside the timed
region), the FP64 CPU oracle timed on a bounded sample of the same workload,
the estimator's health on that workload (ESS, Picard residuals), the
surrogate-vs-plain study at equal RMS value error, the uneven-batch study
(one batched graph vs one call per problem), the flock study (hash-grid
7-NN search and the per-agent sweep over 100,000 agents) and the paper's own
45-dimensional pursuit game (Table 2) timed next to its single-core numbers.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "query·samples/s for v,∇v at n=45; surrogate vs plain MC at equal RMS error"

# Chip figures used for the roofline (MI355X, gfx950).  The FP32 vector peak,
# 157.3 TFLOP/s, is 2 flops per FMA on 256 CUs x 128 lanes x 2.4 GHz: 7.86e13
# full-rate lane operations per second (FMA, MUL, ADD, logic).  Measured on
# this chip: min/max/min3, DPP operands and conversions issue at half that
# rate and transcendentals (sqrt, exp2) at a quarter.
CUS, LANE_SLOTS_PER_CLK, CLOCK_HZ = 256, 128, 2.4e9
VALU_PEAK = CUS * LANE_SLOTS_PER_CLK * CLOCK_HZ     # 7.86e13 full-rate lane-op slots / s


def alu_slots_per_pair(datum: str, n: int) -> int:
    """Minimum full-rate VALU lane-op slots per (query, sample) pair outside the
    dense contractions, for the stacked-disc datum with m = n/3 pairs.

    y = x + theta + sigma z on the 2m planar coordinates -> 2m FMA; |y_k|^2 ->
    m (MUL + FMA); the minimum over m values -> m - 1 compares (two per min3,
    which issues at half rate: one slot per compare); sqrt (4 slots) and the
    radius -> 5; the log-weight a = -c l + (a0 - <z, theta>) -> 2; running
    maximum -> 1; exp2(a - m) -> 1 + 4; S += w, S2 += w^2 -> 2.  Total
    5m + 14.  The two contractions <z, theta> and sum w z (2n MACs) run on the
    matrix cores and are not counted.
    """
    if datum == "min_pair_disks":
        return 5 * (n // 3) + 14
    raise ValueError(datum)


def alu_slots_knn_pair(k: int, n: int) -> int:
    """Minimum full-rate VALU lane-op slots per pair for the flock datum (k
    neighbour balls).

    y on the 3 position coordinates -> 3 FMA; per neighbour 3 SUB, MUL + 2 FMA
    -> 6k, the minimum over k -> k - 1 compares; sqrt (4 slots) and the radius
    -> 5; a -> 2; running maximum -> 1; exp2 -> 5; S, S2 -> 2.  At n = 6 the
    pair loop runs on the vector ALUs, so the two contractions <z, theta> and
    sum w z (2n FMA) count too: 7k + 17 + 2n.
    """
    return 7 * k + 17 + 2 * n


PROFILE = os.path.join(ROOT, "profiles", "pair_loop_dubins15_n45.md")
KERNEL_SOURCES = ["sweep_pairs.h", "sweep_mfma.h", "sweep_impl.h", "kernels.h", "device.h"]


def measured_traffic():
    """HBM bytes per pair-loop launch from the committed counter profile, or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    import re
    if not os.path.exists(PROFILE):
        return None
    text = open(PROFILE).read()
    mt = re.search(r"traffic-bytes-per-launch:\s*(\d+)", text)
    mh = re.search(r"source-hash:\s*([0-9a-f]+)", text)
    if not (mt and mh):
        return None
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2605_18566_amd", "csrc", name), "rb").read())
    return int(mt.group(1)) if h.hexdigest()[:16] == mh.group(1) else None


def _interp_ms_at_rms(points, target):
    """Wall time at RMS = target by log-log interpolation along a series of
    (rms, ms) points ordered by sample count; None if the target is not
    bracketed (the first point already below it counts as reaching it)."""
    import math
    pts = [(r, t) for r, t in points if r > 0 and t > 0]
    for (r0, t0), (r1, t1) in zip(pts, pts[1:]):
        if (r0 - target) * (r1 - target) <= 0 and r0 != r1:
            a = (math.log(target) - math.log(r0)) / (math.log(r1) - math.log(r0))
            return math.exp(math.log(t0) + a * (math.log(t1) - math.log(t0)))
    if pts and pts[0][0] <= target:
        return pts[0][1]
    return None


def surrogate_study(ctx, stream, w, judge_Ks=(5,), cv_modes=(False, True), tols=(1e-3, 1e-2)):
    """Surrogate-accelerated vs plain sweep at equal RMS value error on workload w.

    The network (n+1 -> 4 x 256 SiLU -> n+1) is trained on 2M (x, t) labels of
    the plain sweep (10 horizons t = 0.1 .. 1, 200,000 states each, the
    workload's N and K).  A judge is the plain sweep at N = 2^20 with K in
    judge_Ks iterations and another seed, on the workload's 262,144 states at
    t = 1 (the first is the primary one; every RMS is given against each).  Plain mode: N = 2^12 .. 2^18 at the workload's K.  Surrogate mode:
    N_s = 2^12, 2^14, 2^16, K_s = 1, 2, fallback tolerance in tols, with and
    without the control variate (grad_cv: the Stein gradient's weighted mean
    minus the draws' mean), fallback by the plain sweep at the workload's N and
    K.  RMS of v (and of the gradient's norm) against the judge; wall time per
    sweep (median of 2 after one warm-up, synchronised), network inference
    and fallback included.  Equal RMS: each series' time at the RMS of the
    plain sweep at the workload's N, by log-log interpolation over its sample
    counts.
    """
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import ProblemSpec, Surrogate, TrainConfig, picard_sweep, surrogate_sweep

    f = w.problem_fields()
    dev = torch.device("cuda:0")

    def timed(fn, reps=2):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return r, float(np.median(ts))

    t0 = time.perf_counter()
    xs, ts, vs, gs = [], [], [], []
    horizons, per_h = 10, 200000
    for j in range(horizons):
        tj = (j + 1) / horizons
        x = torch.from_numpy(np.ascontiguousarray(workloads.queries(w, Q=per_h, trial=100 + j).T)).to(dev)
        o = picard_sweep(ctx, ProblemSpec(**dict(f, seed=f["seed"] + 1000 + j)), x, tj, w.N, w.K, time_step=j,
                         stream=stream)
        xs.append(x)
        ts.append(torch.full((per_h,), tj, device=dev))
        vs.append(o.v.clone())
        gs.append(o.grad.clone())
    X, T = torch.cat(xs, 1).contiguous(), torch.cat(ts).contiguous()
    V, G = torch.cat(vs).contiguous(), torch.cat(gs, 1).contiguous()
    torch.cuda.synchronize()
    t_labels = time.perf_counter() - t0
    sur = Surrogate(ctx, w.n, 256, 4, seed=7)
    t0 = time.perf_counter()
    cfg = TrainConfig(epochs=40, batch=4096, lr=2e-3, lr_min=1e-5, weight_decay=1e-4, grad_weight=0.5, seed=11)
    hist = sur.train(X, T, V, G, cfg, stream=stream)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del X, T, V, G, xs, ts, vs, gs
    print(f"surrogate [{w.name}] trained: labels {t_labels:.1f} s, training {t_train:.1f} s, loss {hist[0]:.3f} -> "
          f"{hist[-1]:.3f}", file=sys.stderr, flush=True)

    x = torch.from_numpy(np.ascontiguousarray(workloads.queries(w).T)).to(dev)
    judges = []
    for Kj in judge_Ks:
        t0 = time.perf_counter()
        judge = picard_sweep(ctx, ProblemSpec(**dict(f, seed=f["seed"] + 777)), x, w.t, 1 << 20, Kj, time_step=3,
                             stream=stream)
        torch.cuda.synchronize()
        judges.append({"K": Kj, "v": judge.v.clone(), "g": judge.grad.clone(), "seconds": time.perf_counter() - t0,
                       "resid_hist": [float(r) for r in judge.resid_hist]})

    def errs(v, g):
        """RMS of v and of the gradient's norm against each judge: {"K<k>": (rms_v, rms_grad)}."""
        return {f"K{j['K']}": (float(torch.sqrt(torch.mean((v - j["v"]) ** 2))),
                               float(torch.sqrt(torch.mean(torch.sum((g - j["g"]) ** 2, 0))))) for j in judges}
    jk = [f"K{k}" for k in judge_Ks]
    sv, sg = sur.predict(x, w.t)
    plain, surr = [], []
    for cv in cv_modes:
        spec = ProblemSpec(**dict(f, grad_cv=cv))
        for N in (1 << 12, 1 << 14, 1 << 16, 1 << 18):
            o, sec = timed(lambda: picard_sweep(ctx, spec, x, w.t, N, w.K, stream=stream))
            e = errs(o.v, o.grad)
            plain.append({"N": N, "K": w.K, "grad_cv": cv, "rms_v": {k: e[k][0] for k in jk},
                          "rms_grad": {k: e[k][1] for k in jk}, "ms": sec * 1e3})
    for cv in cv_modes:
        spec = ProblemSpec(**dict(f, grad_cv=cv))
        for tol in tols:
            for K_s in (1, 2):
                for N in (1 << 12, 1 << 14, 1 << 16):
                    (v, g, fb, nfb), sec = timed(lambda: surrogate_sweep(ctx, sur, spec, x, w.t, N, K_s, w.N, w.K,
                                                                         tol, stream=stream))
                    e = errs(v, g)
                    surr.append({"N_s": N, "K_s": K_s, "tol": tol, "grad_cv": cv, "rms_v": {k: e[k][0] for k in jk},
                                 "rms_grad": {k: e[k][1] for k in jk}, "ms": sec * 1e3, "fallback": nfb / w.Q})
    print(f"surrogate [{w.name}] sweeps done", file=sys.stderr, flush=True)
    ref = next(r for r in plain if r["N"] == w.N and not r["grad_cv"])
    big = next(r for r in plain if r["N"] == 4 * w.N and not r["grad_cv"])
    equal = {}
    for k in jk:
        target, target_4n = ref["rms_v"][k], big["rms_v"][k]
        rows_k = []
        for cv in cv_modes:
            series = [(r["rms_v"][k], r["ms"]) for r in plain if r["grad_cv"] == cv]
            ms = _interp_ms_at_rms(series, target)
            rows_k.append({"mode": "plain", "grad_cv": cv, "ms_at_target": ms,
                           "speedup": (ref["ms"] / ms) if ms else None})
            for tol in tols:
                for K_s in (1, 2):
                    rows = [r for r in surr if r["grad_cv"] == cv and r["tol"] == tol and r["K_s"] == K_s]
                    ms = _interp_ms_at_rms([(r["rms_v"][k], r["ms"]) for r in rows], target)
                    ms4 = _interp_ms_at_rms([(r["rms_v"][k], r["ms"]) for r in rows], target_4n)
                    rows_k.append({"mode": "surrogate", "grad_cv": cv, "tol": tol, "K_s": K_s, "ms_at_target": ms,
                                   "speedup": (ref["ms"] / ms) if ms else None,
                                   "speedup_vs_plain_4N": (big["ms"] / ms4) if ms4 else None,
                                   "best_rms_v": min(r["rms_v"][k] for r in rows),
                                   "fallback_range": [min(r["fallback"] for r in rows),
                                                      max(r["fallback"] for r in rows)]})
        equal[f"judge_{k}"] = {"target_rms_v": target, "target_rms_v_plain_4N": target_4n, "table": rows_k}
    sur.close()
    e_alone = errs(sv, sg)
    return {"workload": f"{w.name}: n={w.n}, H={w.ham}{' (tube)' if w.tube else ''}, {w.datum}, nu={w.nu}, "
                        f"t={w.t}, bf16 draws, Q={w.Q}",
            "network": f"{w.n + 1} -> 4 x 256 SiLU -> {w.n + 1}, bf16 MFMA forward/backward, fp32 master, AdamW",
            "training": {"labels": horizons * per_h, "label_N": w.N, "label_K": w.K, "epochs": cfg.epochs,
                         "label_seconds": t_labels, "train_seconds": t_train, "loss_first": float(hist[0]),
                         "loss_last": float(hist[-1])},
            "judges": [{"N": 1 << 20, "K": j["K"], "seed_offset": 777, "seconds": j["seconds"],
                        "resid_hist": j["resid_hist"]} for j in judges],
            "surrogate_alone": {k: {"rms_v": e_alone[k][0], "rms_grad": e_alone[k][1]} for k in jk},
            "plain": plain, "surrogate": surr, "target_ms": ref["ms"], "equal_rms": equal}


def batched_study(ctx, stream, P: int = 256):
    """The uneven batch (stacked Dubins pairs, n = 3..48, N and Q log-uniform,
    K = 3..8): one call per problem vs one batched call (one recorded graph),
    before and after the autotuner picks the samples per split."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import ProblemSpec, autotune_batched, picard_sweep, picard_sweep_batched
    batch = workloads.c3_batch(P=P)
    dev = torch.device("cuda:0")
    xs = [torch.from_numpy(np.ascontiguousarray(workloads.queries(bp.w, trial=1 + i).T)).to(dev)
          for i, bp in enumerate(batch)]
    specs = []
    for bp in batch:
        f = workloads.c3_fields(bp)
        specs.append(ProblemSpec(problem_id=bp.problem_id, **f))
    N = [bp.w.N for bp in batch]
    K = [bp.w.K for bp in batch]
    t = [bp.w.t for bp in batch]
    pairs = float(sum(bp.w.Q * bp.w.N * bp.w.K for bp in batch))

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    with torch.cuda.stream(stream):
        def one_by_one():
            for p in range(P):
                picard_sweep(ctx, specs[p], xs[p], t[p], N[p], K[p], host_outputs=False, stream=stream)
        one_by_one()                                            # records the per-problem graphs
        dt_one, _ = timed(one_by_one)
        print(f"batched study: one call per problem {dt_one:.3f} s", file=sys.stderr, flush=True)

        def batched():
            return picard_sweep_batched(ctx, specs, xs, N, K, t, host_outputs=False, stream=stream)
        batched()                                               # records the batched graph
        dt_b, _ = timed(batched)
        print(f"batched study: one batched call {dt_b:.3f} s", file=sys.stderr, flush=True)
        split, _ = autotune_batched(ctx, specs, xs, N, K, t, stream=stream)
        with tempfile.TemporaryDirectory() as tmp:
            ctx.save_tuning(os.path.join(tmp, "tuning.txt"))
            table = dict(line.split(" = ") for line in open(os.path.join(tmp, "tuning.txt")).read().splitlines()[1:])
        mode = int(table.get("batch_mode", "4")) - 1
        batched()
        dt_t, out = timed(batched)
        print(f"batched study: tuned split {split}, launch mode {mode}: {dt_t:.3f} s", file=sys.stderr, flush=True)
    v = out.v.cpu().numpy()
    if not np.all(np.isfinite(v)):
        raise RuntimeError("non-finite values in the batched study")
    ns = [bp.w.n for bp in batch]
    slots = float(sum(bp.w.Q * bp.w.N * bp.w.K * alu_slots_per_pair(bp.w.datum, bp.w.n) for bp in batch))
    return {"workload": f"{P} uneven problems: n = 3m, m ~ U{{1..16}} (n {min(ns)}..{max(ns)}), "
                        "N log-U[4096, 262144], Q log-U[1024, 65536], nu log-U[1e-3, 1e-1], K ~ U{3..8}, "
                        "bf16 common draws, tube coefficient, Laplace shift",
            "pairs": pairs,
            "one_call_per_problem": {"seconds": dt_one, "query_samples_per_s": pairs / dt_one},
            "batched_default_split": {"seconds": dt_b, "query_samples_per_s": pairs / dt_b},
            "batched_autotuned": {"samples_per_split": split, "persistent": bool(mode & 1),
                                  "concurrent_branches": bool(mode & 2), "seconds": dt_t,
                                  "query_samples_per_s": pairs / dt_t},
            "speedup_batched_vs_one_by_one": dt_one / dt_t,
            "alu_frac_whole_call": slots / dt_t / VALU_PEAK,
            "one_call_per_problem_includes": "per-call table generation and graph recording (16-graph cache)"}


def batched_headline(steps: int):
    """The headline problem alone through the batched path (P = 1) and through
    the single-problem path, `steps` timed calls each after one recording call:
    for comparing the two pair-loop kernels on the same work in one trace."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import Context, ProblemSpec, picard_sweep, picard_sweep_batched
    w = workloads.C5
    x = torch.from_numpy(np.ascontiguousarray(workloads.queries(w, trial=1).T)).to(torch.device("cuda:0"))
    spec = ProblemSpec(**w.problem_fields())
    ctx = Context(0)
    calls = {"single": lambda: picard_sweep(ctx, spec, x, w.t, w.N, w.K, host_outputs=False),
             "batched": lambda: picard_sweep_batched(ctx, [spec], [x], [w.N], [w.K], [w.t], host_outputs=False)}
    secs = {}
    for name, call in calls.items():
        call()
        torch.cuda.synchronize()
        secs[name] = []
        for _ in range(steps):
            t0 = time.perf_counter()
            call()
            torch.cuda.synchronize()
            secs[name].append(time.perf_counter() - t0)
    ctx.close()
    return {"workload": f"{w.name} alone, batched path (P = 1) and single-problem path",
            "seconds": secs, "batch_split": os.environ.get("HJG_BATCH_SPLIT", "default")}


def knn_only(steps: int):
    """The 100,000-agent flock's 7-NN grid search alone, `steps` calls after
    one untimed call: for kernel traces and counters of the search."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import Context, knn_grid
    w = workloads.C4
    st = workloads.flock_agents(w.Q, trial=0)
    pos = torch.from_numpy(np.ascontiguousarray(st[:, :3].T)).to(torch.device("cuda:0"))
    ext, k = workloads.FLOCK_EXTENT, int(w.datum_p[1])
    ctx = Context(0)
    idx, nbr = knn_grid(ctx, pos, (0, 0, 0), (ext,) * 3, workloads.FLOCK_CELL, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        knn_grid(ctx, pos, (0, 0, 0), (ext,) * 3, workloads.FLOCK_CELL, k, want_idx=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / max(steps, 1) * 1e3
    i64 = idx.cpu().numpy().astype(np.int64)
    ctx.close()
    return {"workload": f"{w.name}: {w.Q} agents, {k}-NN grid search", "ms_per_call": ms,
            "idx_sum": int(i64.sum()), "nbr_sum": float(nbr.double().sum())}


def batched_only(steps: int):
    """The uneven batch alone: one recording call, then `steps` timed calls of
    the batched sweep (no other work), for per-kernel profiles."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import Context, ProblemSpec, picard_sweep_batched
    batch = workloads.c3_batch(P=256)
    dev = torch.device("cuda:0")
    xs = [torch.from_numpy(np.ascontiguousarray(workloads.queries(bp.w, trial=1 + i).T)).to(dev)
          for i, bp in enumerate(batch)]
    specs = [ProblemSpec(problem_id=bp.problem_id, **workloads.c3_fields(bp)) for bp in batch]
    N, K, t = [bp.w.N for bp in batch], [bp.w.K for bp in batch], [bp.w.t for bp in batch]
    ctx = Context(0)
    picard_sweep_batched(ctx, specs, xs, N, K, t, host_outputs=False)
    torch.cuda.synchronize()
    secs = []
    for _ in range(steps):
        t0 = time.perf_counter()
        picard_sweep_batched(ctx, specs, xs, N, K, t, host_outputs=False)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
    pairs = float(sum(bp.w.Q * bp.w.N * bp.w.K for bp in batch))
    ctx.close()
    return {"workload": "c3 uneven batch (256 problems)", "pairs": pairs, "seconds": secs,
            "query_samples_per_s": pairs / min(secs),
            "concurrent_branches": os.environ.get("HJG_BATCH_CONCURRENT", "default")}


def dint_study(ctx, stream):
    """The paper's double integral plant at its convergence table's setting:
    x1' = x2, x2' = u, |u| <= 1, H = p1 x2 - |p2| (the minimising control),
    disc of radius 0.2 about the origin, delta = 0.08, N = 8,000 fresh draws
    per state and iteration, K = 15, on a 128 x 128 grid of [-1, 1]^2; the
    table's backward times 0.8, 0.5, 0.2, 0.0 read as horizons 1 - t.  Final
    relative L2 residual and wall time of each sweep (one graph replay,
    synchronised), plain estimator and with the Laplace shift."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import ProblemSpec, picard_sweep
    w = workloads.C9
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.ascontiguousarray(workloads.dint_grid(128).T)).to(dev)
    paper = {0.8: 0.0143, 0.5: 0.0334, 0.2: 0.0596, 0.0: 0.0828}
    runs = {}
    for tilt in (False, True):
        spec = ProblemSpec(**dict(w.problem_fields(), tilt=tilt))
        rows = []
        for tp in workloads.DINT_TIMES:
            tau = 1.0 - tp
            picard_sweep(ctx, spec, x, tau, w.N, w.K, stream=stream)      # records the graph
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = picard_sweep(ctx, spec, x, tau, w.N, w.K, stream=stream)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            v = o.v.cpu().numpy()
            rows.append({"paper_t": tp, "horizon": tau, "iterations": o.iters_done,
                         "final_residual": float(o.resid_hist[-1]), "paper_final_residual": paper[tp],
                         "residual_hist": [float(r) for r in o.resid_hist], "seconds": sec,
                         "query_samples_per_s": w.Q * w.N * w.K / sec, "frac_v_le_0": float(np.mean(v <= 0))})
        runs["laplace_shift" if tilt else "plain"] = rows
    return {"workload": f"{w.name}: 128 x 128 grid of [-1, 1]^2, H = p1 x2 - |p2|, disc r = 0.2 about the origin, "
                        f"nu = {w.nu} (delta = 0.08), N = {w.N} fresh draws, K = {w.K}",
            "runs": runs,
            "note": "the paper gives neither the target radius nor its evaluation states; its table lists backward "
                    "times 0.8 .. 0.0, read here as horizons 0.2 .. 1.0 (a horizon of 0 leaves v = l exactly)"}


def flock_study(ctx, stream):
    """The 100,000-agent flock: hash-grid 7-NN search, then the Picard sweep
    (K = 3, N = 4,096 bf16 common draws) at the 5 horizons t_j = 0.2 j."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import ProblemSpec, knn_grid, picard_sweep
    w = workloads.C4
    dev = torch.device("cuda:0")
    st = workloads.flock_agents(w.Q, trial=0)
    pos = torch.from_numpy(np.ascontiguousarray(st[:, :3].T)).to(dev)
    x = torch.from_numpy(np.ascontiguousarray(st.T)).to(dev)
    ext = workloads.FLOCK_EXTENT
    k = int(w.datum_p[1])
    with torch.cuda.stream(stream):
        _, nbr = knn_grid(ctx, pos, (0, 0, 0), (ext,) * 3, workloads.FLOCK_CELL, k, want_idx=False, stream=stream)
        reps = 20
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            knn_grid(ctx, pos, (0, 0, 0), (ext,) * 3, workloads.FLOCK_CELL, k, want_idx=False, stream=stream)
        torch.cuda.synchronize()
        knn_ms = (time.perf_counter() - t0) / reps * 1e3
        spec = ProblemSpec(datum_aux=nbr, **w.problem_fields())
        hs = workloads.horizons(w)

        def sweep_all(out=None):
            outs = []
            for j, t in enumerate(hs):
                outs.append(picard_sweep(ctx, spec, x, t, w.N, w.K, time_step=j + 1, host_outputs=False,
                                         stream=stream))
            return outs
        sweep_all()                                        # records one graph per horizon
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = sweep_all()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.set_timing(True)
        kernel_ms, launches = 0.0, 0
        for j, t in enumerate(hs):
            picard_sweep(ctx, spec, x, t, w.N, w.K, time_step=j + 1, host_outputs=False, stream=stream)
            ms, nl = ctx.sweep_time()
            kernel_ms += ms
            launches += nl
        ctx.set_timing(False)
        last = picard_sweep(ctx, spec, x, hs[-1], w.N, w.K, time_step=len(hs), stream=stream)
        # population certification at the last horizon: the plain estimator
        # (the concentration theorems' setting) and its per-agent sampling
        # margin at confidence 0.95 (l >= -r; no upper bound), Hoeffding and
        # the variance-aware empirical Bernstein form
        from paper_2605_18566_amd import certify, mc_margin
        plain = ProblemSpec(datum_aux=nbr, **dict(w.problem_fields(), tilt=False))
        pc = picard_sweep(ctx, plain, x, hs[-1], w.N, w.K, time_step=len(hs), host_outputs=False, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        marg = mc_margin(pc.v, pc.c, w.N, 0.05, -float(w.datum_p[0]), ess=pc.ess, stream=stream)
        lab, cnt = certify(pc.v, 0.0, marg, stream=stream)
        torch.cuda.synchronize()
        cert_ms = (time.perf_counter() - t0) * 1e3
        marg_h = mc_margin(pc.v, pc.c, w.N, 0.05, -float(w.datum_p[0]), stream=stream)
        _, cnt_h = certify(pc.v, 0.0, marg_h, stream=stream)
    cnt, cnt_h = cnt.cpu().numpy(), cnt_h.cpu().numpy()
    mg, mgh = marg.cpu().numpy(), marg_h.cpu().numpy()

    def _med(a):
        return float(np.median(a[np.isfinite(a)])) if np.isfinite(a).any() else None
    certification = {"estimator": "plain (no shift), tube coefficient, last horizon, K = 3",
                     "confidence": 0.95,
                     "bernstein": {"unsafe": int(cnt[0]), "undetermined": int(cnt[1]), "safe": int(cnt[2]),
                                   "certified_fraction": float((cnt[0] + cnt[2]) / w.Q),
                                   "finite_margin_fraction": float(np.mean(np.isfinite(mg))),
                                   "median_finite_margin": _med(mg)},
                     "hoeffding": {"unsafe": int(cnt_h[0]), "undetermined": int(cnt_h[1]), "safe": int(cnt_h[2]),
                                   "certified_fraction": float((cnt_h[0] + cnt_h[2]) / w.Q),
                                   "finite_margin_fraction": float(np.mean(np.isfinite(mgh))),
                                   "median_finite_margin": _med(mgh)},
                     "margin_and_labels_ms": cert_ms,
                     "budget": "sampling term only (per agent); the iteration, quasi-linearisation and viscosity "
                               "terms need constants the paper does not evaluate and are taken as 0"}
    v = torch.stack([o.v for o in outs]).cpu().numpy()
    if not np.all(np.isfinite(v)):
        raise RuntimeError("non-finite values in the flock study")
    pairs = float(w.Q * w.N * w.K * len(hs))
    slots = alu_slots_knn_pair(k, w.n)
    per_launch = kernel_ms / max(launches, 1)
    achieved = slots * w.Q * w.N / (per_launch * 1e-3)
    # algorithmic bytes of build + search: positions read twice (24), cell
    # ids and ranks written and read (16), cell-ordered records written and
    # read (32), k neighbour indices and positions written (16k)
    knn_bytes = w.Q * (24 + 16 + 32 + 16 * k)
    return {"workload": f"{w.name}: {w.Q} agents, 7-NN union-of-balls target (r = 0.2), double integrator, "
                        f"nu = {w.nu}, {len(hs)} horizons x K = {w.K}, N = {w.N} bf16 common draws, tube coefficient",
            "knn_grid_ms": knn_ms,
            "knn_grid_algorithmic_GBps": knn_bytes / (knn_ms * 1e-3) / 1e9,
            "knn_grid_note": "one finiteness check (a stream synchronisation) and six small launches for 100,000 "
                             "agents: latency-bound, far from the 8 TB/s HBM roofline",
            "sweep_seconds_all_horizons": dt,
            "query_samples_per_s": pairs / dt,
            "pair_loop": {"bound": "alu", "alu_slots_per_pair": slots, "kernel_ms_per_launch": per_launch,
                          "achieved_TOPs": achieved / 1e12, "frac": achieved / VALU_PEAK},
            "population_certification": certification,
            "health_last_horizon": {"resid_hist": [float(r) for r in last.resid_hist],
                                    "ess_median": float(np.median(last.ess.cpu().numpy())),
                                    "frac_v_below_zero": float(np.mean(last.v.cpu().numpy() < 0))}}


def small_configs_study(ctx, stream):
    """The two small configurations: C1 (n = 2, fresh draws, one iteration)
    and C2 (n = 3 relative Dubins, 10 horizons x K = 5, N = 65,536 common
    draws), both on the vector-ALU pair loop."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import ProblemSpec, picard_sweep, value_grad
    out = {}
    with torch.cuda.stream(stream):
        w = workloads.C1
        x = torch.from_numpy(np.ascontiguousarray(workloads.queries(w).T)).to("cuda:0")
        spec = ProblemSpec(**w.problem_fields())
        c = torch.full((w.Q,), 1.0 / (2.0 * w.nu), dtype=torch.float32, device="cuda:0")
        value_grad(ctx, spec, x, w.t, w.N, c, stream=stream)
        reps = 20
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            value_grad(ctx, spec, x, w.t, w.N, c, stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out["c1_quadratic_disk_n2"] = {"Q": w.Q, "N": w.N, "K": w.K, "draws": "fresh Philox per query",
                                       "seconds_per_sweep": dt, "query_samples_per_s": w.Q * w.N / dt}
        w = workloads.C2
        x = torch.from_numpy(np.ascontiguousarray(workloads.queries(w).T)).to("cuda:0")
        spec = ProblemSpec(**w.problem_fields())
        hs = workloads.horizons(w)
        for j, t in enumerate(hs):                              # record the graphs
            picard_sweep(ctx, spec, x, t, w.N, w.K, time_step=j + 1, host_outputs=False, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j, t in enumerate(hs):
            picard_sweep(ctx, spec, x, t, w.N, w.K, time_step=j + 1, host_outputs=False, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.set_timing(True)
        picard_sweep(ctx, spec, x, hs[-1], w.N, w.K, time_step=len(hs), host_outputs=False, stream=stream)
        ms, nl = ctx.sweep_time()
        ctx.set_timing(False)
        slots = alu_slots_per_pair(w.datum, w.n) + 2 * w.n      # contractions on the vector ALUs at n = 3
        out["c2_dubins_n3"] = {"Q": w.Q, "N": w.N, "K": w.K, "horizons": len(hs), "seconds_all_horizons": dt,
                               "query_samples_per_s": w.Q * w.N * w.K * len(hs) / dt,
                               "pair_loop": {"kernel_ms_per_launch": ms / max(nl, 1), "alu_slots_per_pair": slots,
                                             "frac": slots * w.Q * w.N / (ms / max(nl, 1) * 1e-3) / VALU_PEAK}}
    return out


def pursuit_study(ctx, stream):
    """The paper's 45-dimensional multi-pursuer single-evader game (Table 2):
    three speed regimes, K = 15 Picard iterations, N = 20,000 draws, 1,600
    states; wall time per regime next to the paper's single-core times."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import ProblemSpec, picard_sweep
    w = workloads.C6
    x = torch.from_numpy(np.ascontiguousarray(workloads.queries(w).T)).to("cuda:0")
    paper_s = {"evader_faster": 12.7, "equal_speed": 12.6, "pursuers_faster": 12.6}
    rows = {}
    with torch.cuda.stream(stream):
        for name, (ae, ap) in workloads.PURSUIT_REGIMES.items():
            spec = ProblemSpec(**dict(w.problem_fields(), ham_p=(ae, ap, 1.0)))
            picard_sweep(ctx, spec, x, w.t, w.N, w.K, stream=stream)           # records the graph
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = picard_sweep(ctx, spec, x, w.t, w.N, w.K, stream=stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rows[name] = {"a_evader": ae, "a_pursuer": ap, "seconds": dt,
                          "query_samples_per_s": w.Q * w.N * w.K / dt,
                          "final_relative_residual": float(out.resid_hist[-1]),
                          "paper_seconds_one_cpu_core": paper_s[name]}
    return {"workload": f"{w.name}: 14 pursuers + 1 evader, n = 45, Q = {w.Q}, N = {w.N} bf16 common draws, "
                        f"K = {w.K}, nu = {w.nu}, capture radius 1.5, tube coefficient, tilt",
            "regimes": rows,
            "note": "the paper does not state its state count or N for this table; 1,600 states and N = 20,000 "
                    "are readings (its 3D slices use 1,600 points; 7.2 MB per iteration at n = 45 is N = 20,000 "
                    "in float64); positions uniform over [-100, 100] per coordinate as the paper states"}


def _march(ctx, w, cfg, spec, xtr, xev, stream, obstacle=None):
    """March the workload over its horizons (semigroup form, surrogate as the
    datum); with an obstacle (ProblemSpec of the avoid set's level) every
    step's labels and the final values are projected onto the reach-avoid
    constraint.  Returns the final step at xev, its warm time and the march
    timings."""
    import torch

    from paper_2605_18566_amd import Surrogate, TrainConfig, avoid_project, picard_sweep, surrogate_tube_step
    dt = w.T / w.time_steps
    M = xtr.shape[1]
    sur = Surrogate(ctx, w.n, cfg["width"], cfg["depth"], seed=5)
    tc = dict(epochs=cfg["epochs"], batch=cfg["batch"], lr=cfg["lr"], lr_min=cfg["lr_min"])

    def lift(x, o):
        if obstacle is not None:
            avoid_project(obstacle, x, o.v, o.grad, stream=stream)
        return o

    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        first = lift(xtr, picard_sweep(ctx, spec, xtr, dt, cfg["N"], cfg["K"], time_step=1, host_outputs=False,
                                       stream=stream))
        lx, lt, lv, lg = [xtr], [torch.full((M,), dt, device="cuda:0")], [first.v.clone()], [first.grad.clone()]
        train_s = step_s = 0.0
        for j in range(2, w.time_steps + 1):
            torch.cuda.synchronize()
            a = time.perf_counter()
            sur.train(torch.cat(lx, 1).contiguous(), torch.cat(lt).contiguous(), torch.cat(lv).contiguous(),
                      torch.cat(lg, 1).contiguous(), TrainConfig(seed=j, **tc), stream=stream)
            torch.cuda.synchronize()
            b = time.perf_counter()
            o = lift(xtr, surrogate_tube_step(ctx, sur, spec, xtr, (j - 1) * dt, dt, cfg["N"], cfg["K"], time_step=j,
                                              stream=stream))
            torch.cuda.synchronize()
            train_s += b - a
            step_s += time.perf_counter() - b
            lx.append(xtr)
            lt.append(torch.full((M,), j * dt, device="cuda:0"))
            lv.append(o.v.clone())
            lg.append(o.grad.clone())
        march_s = time.perf_counter() - t0
        # the last step at the evaluation states, timed warm
        args = (ctx, sur, spec, xev, w.T - dt, dt, cfg["N"], cfg["K"])
        surrogate_tube_step(*args, time_step=w.time_steps, stream=stream)
        torch.cuda.synchronize()
        a = time.perf_counter()
        ev = lift(xev, surrogate_tube_step(*args, time_step=w.time_steps, stream=stream))
        torch.cuda.synchronize()
        ev_s = time.perf_counter() - a
    sur.close()
    return ev, ev_s, march_s, train_s, step_s


def tube_study(ctx, stream):
    """Time marching with the surrogate as the datum (semigroup form): march
    the n = 3 Dubins tube workload and the exact quadratic case over ten
    horizons, compare with the direct horizon sweep (and, for the quadratic
    case, with its closed form), and time the last step at 65,536 states."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import ProblemSpec, picard_sweep
    cfg = workloads.TUBE_MARCH
    res = {}
    for w in (workloads.C2, workloads.Q3):
        spec = ProblemSpec(**w.problem_fields())
        dt = w.T / w.time_steps
        M = cfg["train_states"]
        xtr = torch.from_numpy(np.ascontiguousarray(workloads.queries(w, Q=M, trial=7).T)).to("cuda:0")
        xev = torch.from_numpy(np.ascontiguousarray(workloads.queries(w).T)).to("cuda:0")
        ev, ev_s, march_s, train_s, step_s = _march(ctx, w, cfg, spec, xtr, xev, stream)
        with torch.cuda.stream(stream):
            direct = picard_sweep(ctx, spec, xev, w.T, w.N, w.K, time_step=w.time_steps, host_outputs=False,
                                  stream=stream)
            torch.cuda.synchronize()
        vm, vd = ev.v.cpu().numpy(), direct.v.cpu().numpy()
        rows = w.Q * cfg["N"] * ev.iters_done
        nin, wd, dp = w.n + 1, cfg["width"], cfg["depth"]
        macs = nin * wd + (dp - 1) * wd * wd + wd * nin
        r = {"states": w.Q, "samples": cfg["N"], "picard_iterations": ev.iters_done, "dt": dt,
             "last_step_seconds": ev_s, "network_rows_per_s": rows / ev_s,
             "network_tflops": 2.0 * macs * rows / ev_s / 1e12,
             "mfma_frac": 2.0 * macs * rows / ev_s / 2.5e15,
             "march_seconds": march_s, "training_seconds": train_s, "label_step_seconds": step_s,
             "marched_vs_direct_rms": float(np.sqrt(np.mean((vm - vd) ** 2))),
             "direct_rms": float(np.sqrt(np.mean(vd ** 2))),
             "sign_agreement": float(np.mean(np.sign(vm) == np.sign(vd))),
             "inside_fraction_marched": float(np.mean(vm <= 0)), "inside_fraction_direct": float(np.mean(vd <= 0))}
        if w.ham == "quadratic":
            x = xev.cpu().numpy().astype(np.float64)
            exact = np.sum(x * x, 0) / (2 * (1 + w.T)) + w.n * w.nu * np.log1p(w.T)
            r["marched_vs_exact_rms"] = float(np.sqrt(np.mean((vm - exact) ** 2)))
            r["direct_vs_exact_rms"] = float(np.sqrt(np.mean((vd - exact) ** 2)))
            r["exact_rms"] = float(np.sqrt(np.mean(exact ** 2)))
        res[w.name] = r
    return {"workload": f"ten horizons t_j = 0.1 j; labels on {cfg['train_states']} training states per step "
                        f"(N = {cfg['N']}, K = {cfg['K']}); network {cfg['depth']} x {cfg['width']} SiLU trained "
                        f"{cfg['epochs']} epochs per step on all labels so far; last step at the workload's states; "
                        "direct = Algorithm 1 at the final horizon from the terminal datum",
            "runs": res}


def reach_avoid_study(ctx, stream):
    """Reach-avoid tube on the n = 3 Dubins workload: the same march as the
    time-marching study with every step's values projected onto the obstacle
    constraint of two discs in the relative plane, against the plain tube and
    against a projection at the final horizon only; then the projection
    kernel alone at 2^23 states (HBM roofline)."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import ProblemSpec, avoid_project
    w, cfg = workloads.C2, workloads.TUBE_MARCH
    spec = ProblemSpec(**w.problem_fields())
    cen = torch.tensor(workloads.AVOID_DISCS, dtype=torch.float32, device="cuda:0")
    obst = ProblemSpec(n=w.n, datum="disc_union", datum_p=(workloads.AVOID_RADIUS, len(workloads.AVOID_DISCS)),
                       datum_aux=cen)
    xtr = torch.from_numpy(np.ascontiguousarray(workloads.queries(w, Q=cfg["train_states"], trial=7).T)).to("cuda:0")
    xev = torch.from_numpy(np.ascontiguousarray(workloads.queries(w).T)).to("cuda:0")
    plain, *_ = _march(ctx, w, cfg, spec, xtr, xev, stream)
    ra, ev_s, march_s, train_s, step_s = _march(ctx, w, cfg, spec, xtr, xev, stream, obstacle=obst)
    with torch.cuda.stream(stream):
        final_only_v = plain.v.clone()
        act = avoid_project(obst, xev, final_only_v, None, want_active=True, stream=stream)
        torch.cuda.synchronize()
    x = xev.cpu().numpy().astype(np.float64)
    c = workloads.AVOID_DISCS
    lvl = np.min([np.hypot(x[0] - a, x[1] - b) for a, b in c], axis=0) - workloads.AVOID_RADIUS
    inside = lvl < 0
    vp, vr, vf = plain.v.cpu().numpy(), ra.v.cpu().numpy(), final_only_v.cpu().numpy()
    res = {"states": w.Q, "avoid_fraction_of_states": float(np.mean(inside)),
           "inside_fraction_tube": float(np.mean(vp <= 0)),
           "inside_fraction_final_projection": float(np.mean(vf <= 0)),
           "inside_fraction_reach_avoid": float(np.mean(vr <= 0)),
           "avoid_states_reached_tube": int(np.sum(inside & (vp <= 0))),
           "avoid_states_reached_reach_avoid": int(np.sum(inside & (vr <= 0))),
           "reached_only_through_the_obstacle": int(np.sum((vf <= 0) & (vr > 0))),
           "final_projection_active": float(act.float().mean().item()),
           "march_seconds": march_s, "training_seconds": train_s, "label_step_seconds": step_s,
           "last_step_seconds": ev_s}
    # the projection kernel alone, 2^23 states, fresh values for every timed call
    Q, reps = 1 << 23, 8
    g = torch.Generator(device="cuda:0").manual_seed(3)
    xb = (torch.rand((w.n, Q), generator=g, device="cuda:0") * 6 - 3).contiguous()
    vs = [(torch.rand(Q, generator=g, device="cuda:0") * 4 - 2) for _ in range(reps + 1)]
    gs = [torch.zeros((w.n, Q), device="cuda:0") for _ in range(reps + 1)]
    flags = []
    with torch.cuda.stream(stream):
        avoid_project(obst, xb, vs[reps], gs[reps], want_active=True, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(reps):
            flags.append(avoid_project(obst, xb, vs[i], gs[i], want_active=True, stream=stream))
        e1.record(stream)
        torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    active = float(torch.stack([f.float().mean() for f in flags]).mean().item())
    bytes_per = Q * (4 * w.n + 4 + 1) + active * Q * 4 * (w.n + 1)
    res["projection_kernel"] = {"states": Q, "active_fraction": active, "us_per_launch": ms * 1e3,
                                "algorithmic_bytes": bytes_per, "hbm_gbs": bytes_per / (ms * 1e-3) / 1e9,
                                "hbm_frac": bytes_per / (ms * 1e-3) / 8e12}
    return {"workload": f"{w.name} marched over ten horizons as in the time-marching study; avoid set = union of "
                        f"discs of radius {workloads.AVOID_RADIUS} about {workloads.AVOID_DISCS} in the relative "
                        "plane (heading free); projection after every step (splitting form)", "result": res}


def topology_study(ctx, stream):
    """Topology markers of the Dubins tube's zero-sublevel set on the slice
    heading = 0 (128 x 128 states over [-3, 3]^2) at the ten horizons, and
    the event rules between consecutive horizons."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import ProblemSpec, isocontour, picard_sweep, topology, topology_events
    w = workloads.C2
    m = 128
    g = np.linspace(-3.0, 3.0, m)
    X, Y = np.meshgrid(g, g)
    xs = np.stack([X.ravel(), Y.ravel(), np.zeros(m * m)]).astype(np.float32)
    x = torch.from_numpy(xs).to("cuda:0")
    spec = ProblemSpec(**w.problem_fields())
    vs = []
    with torch.cuda.stream(stream):
        for j in range(1, w.time_steps + 1):
            o = picard_sweep(ctx, spec, x, w.T * j / w.time_steps, w.N, w.K, time_step=j, host_outputs=False,
                             stream=stream)
            vs.append(o.v.view(m, m))
        v = torch.stack(vs).contiguous()
        topology(v, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nc, b1, chi = topology(v, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        seg, sl = isocontour(v, 0.0, stream=stream)
        seg_len = torch.linalg.vector_norm(seg[:, 2:] - seg[:, :2], dim=1) * (6.0 / (m - 1))
        perimeter = [float(seg_len[sl == j].sum()) for j in range(len(vs))]
    nc, b1, chi = nc.cpu().numpy(), b1.cpu().numpy(), chi.cpu().numpy()
    ev = topology_events(chi, b1, nc)
    names = {1: "vacuole", 2: "cordon", 4: "fragmentation"}
    return {"workload": f"{w.name}: slice heading = 0, {m} x {m} states over [-3, 3]^2, horizons t_j = 0.1 j, "
                        f"N = {w.N}, K = {w.K}",
            "n_comp": nc.tolist(), "beta1": b1.tolist(), "chi": chi.tolist(),
            "inside_fraction": [float((vv <= 0).float().mean()) for vv in vs],
            "events": [[names[b] for b in (1, 2, 4) if e & b] for e in ev.tolist()],
            "zero_level_contour_length": perimeter,
            "zero_level_contour_length_disc": 2 * 3.141592653589793 * 0.5,
            "topology_ms_for_all_slices": ms}


def rockets_study(ctx, stream):
    """The paper's two-rocket game (Table 1 rows "Rockets"): 40 x 40 (x, z)
    slices at the headings -pi/2, 0, pi/2, N = 14,000 fresh draws, K = 12;
    wall time per slice next to the paper's single-core times."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import ProblemSpec, picard_sweep
    w = workloads.C7
    spec = ProblemSpec(**w.problem_fields())
    paper_s = {"-pi/2": 13.5, "0": 13.5, "pi/2": 13.6}
    rows = {}
    with torch.cuda.stream(stream):
        for name, th in zip(("-pi/2", "0", "pi/2"), workloads.ROCKET_HEADINGS):
            x = torch.from_numpy(np.ascontiguousarray(workloads.rocket_slice(th).T)).to("cuda:0")
            picard_sweep(ctx, spec, x, w.t, w.N, w.K, stream=stream)          # records the graph
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = picard_sweep(ctx, spec, x, w.t, w.N, w.K, stream=stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rows[name] = {"seconds": dt, "query_samples_per_s": w.Q * w.N * w.K / dt,
                          "final_relative_residual": float(out.resid_hist[-1]),
                          "inside_fraction": float((out.v <= 0).float().mean()),
                          "paper_seconds_one_cpu_core": paper_s[name]}
    return {"workload": f"{w.name}: relative (x, z, theta), a = 64, g = 32, |u| <= 1, capture radius 1.5, "
                        f"40 x 40 slices of (-100, 100]^2, N = {w.N} fresh draws, K = {w.K}, nu = {w.nu}, "
                        "tube coefficient, plain estimator",
            "headings": rows,
            "note": "the Hamiltonian is derived from the rows of the paper's definition (its simplified form swaps "
                    "u_e and u_p and drops a sign); the paper's residual floor for this game is 0.020-0.062 over "
                    "its own evaluation grid"}


def murmuration_study(ctx, stream):
    """The paper's murmuration study: certify all 99,996 starlings at the end
    of the horizon (each bird's value read at its own 4D state, per-bird
    empirical Bernstein margin), and the topology of the zero-sublevel set on
    the 128 x 128 window at 18 times of the horizon (smoothed by 1.5 cells)."""
    import numpy as np
    import torch

    import workloads
    from paper_2605_18566_amd import (ProblemSpec, certify, mc_margin, picard_sweep, smooth_slices, topology,
                                      topology_events)
    w = workloads.C8
    dev = torch.device("cuda:0")
    cen = torch.from_numpy(workloads.murmuration_centres().ravel()).to(dev)
    spec = ProblemSpec(datum_aux=cen, **w.problem_fields())
    birds = torch.from_numpy(np.ascontiguousarray(workloads.starlings().T)).to(dev)
    win = torch.from_numpy(np.ascontiguousarray(workloads.murmuration_window().T)).to(dev)
    taus = [w.T * (j + 1) / w.time_steps for j in range(w.time_steps)]
    with torch.cuda.stream(stream):
        picard_sweep(ctx, spec, birds, w.T, w.N, w.K, tol=1e-5, stream=stream)        # records the graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pop = picard_sweep(ctx, spec, birds, w.T, w.N, w.K, tol=1e-5, stream=stream)
        marg = mc_margin(pop.v, pop.c, w.N, 0.05, -float(w.datum_p[0]), ess=pop.ess, stream=stream)
        lab, cnt = certify(pop.v, 0.0, marg, stream=stream)
        torch.cuda.synchronize()
        cert_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        vs = []
        for j, tau in enumerate(taus):
            o = picard_sweep(ctx, spec, win, tau, w.N, w.K, tol=1e-5, time_step=j + 1, host_outputs=False,
                             stream=stream)
            vs.append(o.v.view(128, 128))
        sm = smooth_slices(torch.stack(vs).contiguous(), workloads.MURMUR_SMOOTH, stream=stream)
        nc, b1, chi = topology(sm, stream=stream)
        torch.cuda.synchronize()
        topo_s = time.perf_counter() - t0
    cnt = cnt.cpu().numpy()
    nc, b1, chi = nc.cpu().numpy(), b1.cpu().numpy(), chi.cpu().numpy()
    ev = topology_events(chi, b1, nc)
    names = {1: "vacuole", 2: "cordon", 4: "fragmentation"}
    v = pop.v.cpu().numpy()
    return {"workload": f"{w.name}: {w.Q} starlings in {workloads.MURMUR_FLOCKS} flocks, 7 pursuers on a ring of "
                        f"radius {workloads.MURMUR_RING}, capture radius {w.datum_p[0]}, delta = {2 * w.nu:.2f}, "
                        f"N = {w.N} common draws per horizon, K <= {w.K} (tol 1e-5), horizon [0, {w.T}]",
            "population": {"positive_value_fraction": float(np.mean(v > 0)),
                           "certified_safe_fraction": float(cnt[2] / w.Q), "certified_unsafe": int(cnt[0]),
                           "undetermined": int(cnt[1]), "picard_iterations": int(pop.iters_done),
                           "final_relative_residual": float(pop.resid_hist[pop.iters_done - 1]),
                           "seconds_sweep_margins_labels": cert_s, "paper_positive_fraction": 0.877},
            "topology": {"tau": taus, "n_comp": nc.tolist(), "beta1": b1.tolist(), "chi": chi.tolist(),
                         "events": [[names[b] for b in (1, 2, 4) if e & b] for e in ev.tolist()],
                         "seconds_18_slices": topo_s,
                         "paper": "hole (beta1 = 1, chi = 0) through tau = 1.18, closing at 1.29; n_comp = 1"},
            "paper_seconds_whole_study_8_cpu_cores": 429.0}


def cpu_model_name() -> str:
    """The host CPU's model name (/proc/cpuinfo), or the platform's description."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_oracle_baseline(w, per_worker: int, workers: int):
    """Time the FP64 oracle (unchanged) on workers x per_worker queries of the workload."""
    import concurrent.futures as cf
    import multiprocessing as mp
    os.environ["OMP_NUM_THREADS"] = "1"
    t0 = time.perf_counter()
    # forked workers, started before this process touches the GPU
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        futs = [ex.submit(_oracle_chunk, w, per_worker, i) for i in range(workers)]
        for f in futs:
            f.result()
    dt = time.perf_counter() - t0
    pairs = workers * per_worker * w.N * w.K
    return pairs / dt, dt, pairs


def _oracle_chunk(w, q, trial):
    import numpy as np

    import workloads
    from oracle import estimator, model
    x = workloads.queries(w, Q=q, trial=100 + trial).astype(np.float64)
    estimator.picard(model.Problem(**w.problem_fields()), x, w.t, w.N, w.K)
    return q


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--queries", type=int, default=None, help="override Q (default: the workload's 262,144)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the equal-accuracy surrogate study")
    ap.add_argument("--no-batched", action="store_true", help="skip the uneven-batch study")
    ap.add_argument("--no-flock", action="store_true", help="skip the flock study")
    ap.add_argument("--no-pursuit", action="store_true", help="skip the 45-dimensional pursuit-game study")
    ap.add_argument("--no-small", action="store_true", help="skip the C1/C2 small-configuration study")
    ap.add_argument("--no-tube", action="store_true", help="skip the time-marching study")
    ap.add_argument("--no-topology", action="store_true", help="skip the topology-marker study")
    ap.add_argument("--no-reach-avoid", action="store_true", help="skip the reach-avoid tube study")
    ap.add_argument("--no-rockets", action="store_true", help="skip the two-rocket game study")
    ap.add_argument("--no-murmuration", action="store_true", help="skip the murmuration study")
    ap.add_argument("--no-dint", action="store_true", help="skip the double-integrator study")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the uneven batch (one batched call, --steps times after one recording call) "
                         "and print its wall time; for kernel profiles of the batched launches")
    ap.add_argument("--batched-headline", action="store_true",
                    help="run only the headline problem through the batched path (P = 1) and the "
                         "single-problem path, --steps calls each; for comparing the two kernels")
    ap.add_argument("--knn-only", action="store_true",
                    help="run only the flock's k-NN grid search, --steps calls; for kernel traces and counters")
    ap.add_argument("--cpu-queries-per-worker", type=int, default=96)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (counter calibration)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only measure the issue rate of independent float32 FMAs at 1..8 waves per SIMD")
    args = ap.parse_args()
    if args.valu_probe:
        from paper_2605_18566_amd import probe_valu_rate
        rows = []
        forms = {0: "fma acc*s+s (scalar operand)", 1: "fmac acc+=a*b", 2: "mul acc*=a", 3: "fma acc*a+b",
                 4: "fmac acc+=s*a (scalar operand)", 5: "add acc+=s (scalar operand)", 6: "min3 (acc, a, b)",
                 7: "forms 0 and 1 on alternate chains",
                 8: "asm S F S F, independent", 9: "asm S F S F, F reads the S before it",
                 10: "asm S F S F, F reads the S two before it",
                 11: "fmac acc+=a*b at 256 VGPRs", 12: "asm S F S F, F reads the S two before it, at 256 VGPRs"}
        for form, what in forms.items():
            for wps in (1, 2, 4, 8):
                r, ghz = probe_valu_rate(wps, form=form)
                rows.append({"form": what, "waves_per_simd": wps, "instr_per_cu_clock": round(r, 4),
                             "clock_ghz": round(ghz, 4)})
                print(f"{what}, waves/SIMD {wps}: {r:.3f} wave-level VALU instructions per CU-clock at "
                      f"{ghz:.3f} GHz", file=sys.stderr, flush=True)
        print(json.dumps({"valu_probe": rows, "peak_instr_per_cu_clock": 2.0}))
        return
    if args.copy_bytes:
        import torch
        a = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(queries would be split across GPUs with no exchange but a 16-byte residual "
              "all-reduce per iteration).", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import workloads

    if args.batched_only:
        print(json.dumps(batched_only(args.steps)))
        return
    if args.batched_headline:
        print(json.dumps(batched_headline(args.steps)))
        return
    if args.knn_only:
        print(json.dumps(knn_only(args.steps)))
        return

    w = workloads.C5
    if args.queries:
        w = w.resized(Q=args.queries)

    cpu = None
    if not args.no_cpu_baseline:
        workers = min(16, os.cpu_count() or 1)
        rate, dt, pairs = cpu_oracle_baseline(w, args.cpu_queries_per_worker, workers)
        cpu = {"value": rate, "unit": "query·samples/s", "cores": workers, "kind": "oracle",
               "cpu_model": cpu_model_name(),
               "sample": f"{workers * args.cpu_queries_per_worker} queries x N={w.N} x K={w.K} of the same "
                         f"workload ({pairs:.3g} pairs, {dt:.1f} s, one process per core)"}
        print(f"cpu baseline: {rate:.3e} pairs/s on {workers} cores ({dt:.1f} s)", file=sys.stderr, flush=True)

    import torch

    from paper_2605_18566_amd import Context, ProblemSpec, picard_sweep

    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.ascontiguousarray(workloads.queries(w).T)).to(dev)
    spec = ProblemSpec(**w.problem_fields())
    ctx = Context(0)
    ctx.set_timing(True)
    stream = torch.cuda.Stream(device=dev)
    out = None
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            out = picard_sweep(ctx, spec, x, w.t, w.N, w.K, host_outputs=False, out=out, stream=stream)
        torch.cuda.synchronize()
        print("warmup done", file=sys.stderr, flush=True)
        kernel_ms, launches = 0.0, 0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = picard_sweep(ctx, spec, x, w.t, w.N, w.K, host_outputs=False, out=out, stream=stream)
            ms, nl = ctx.sweep_time()
            kernel_ms += ms
            launches += nl
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    v = out.v.cpu().numpy()
    if not np.all(np.isfinite(v)):
        raise RuntimeError("non-finite values in the benchmark output")
    ctx.set_timing(False)
    health = {"resid_hist_last_step": None, "ess_median": float(np.median(out.ess.cpu().numpy())),
              "ess_q10": float(np.quantile(out.ess.cpu().numpy(), 0.1)),
              "coefficient_median_abs": float(np.median(np.abs(out.c.cpu().numpy())))}
    chk = picard_sweep(ctx, spec, x, w.t, w.N, w.K, stream=stream)
    health["resid_hist_last_step"] = [float(r) for r in chk.resid_hist]
    study = study_exact = None
    if not args.no_surrogate:
        # the configured workload (15 stacked Dubins pairs, tube coefficient);
        # its Picard iteration keeps moving by ~0.24 relative per iteration at
        # N = 65,536, so the judge runs 20 iterations
        # (and at the configured K = 5 beside it, which measures Monte-Carlo
        # error at equal Picard depth)
        study = surrogate_study(ctx, stream, workloads.C5, judge_Ks=(20, 5))
        # the exact Cole-Hopf case of the same datum and sizes (H = |p|^2/2)
        study_exact = surrogate_study(ctx, stream, workloads.C5Q, judge_Ks=(5,), cv_modes=(False,))
    bstudy = None
    if not args.no_batched:
        bstudy = batched_study(ctx, stream)
    fstudy = None
    if not args.no_flock:
        fstudy = flock_study(ctx, stream)
    pstudy = None
    if not args.no_pursuit:
        pstudy = pursuit_study(ctx, stream)
    sstudy = None
    if not args.no_small:
        sstudy = small_configs_study(ctx, stream)
    tstudy = None
    if not args.no_tube:
        tstudy = tube_study(ctx, stream)
    rastudy = None
    if not args.no_reach_avoid:
        rastudy = reach_avoid_study(ctx, stream)
    topo = None
    if not args.no_topology:
        topo = topology_study(ctx, stream)
    rstudy = None
    if not args.no_rockets:
        rstudy = rockets_study(ctx, stream)
    mstudy = None
    if not args.no_murmuration:
        mstudy = murmuration_study(ctx, stream)
    dstudy = None
    if not args.no_dint:
        dstudy = dint_study(ctx, stream)

    sec_per_step = (t1 - t0) / args.steps
    pairs_per_step = w.Q * w.N * w.K
    value = pairs_per_step / sec_per_step
    slots = alu_slots_per_pair(w.datum, w.n)
    per_launch_ms = kernel_ms / max(launches, 1)
    achieved = slots * w.Q * w.N / (per_launch_ms * 1e-3)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "query·samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: plain Monte-Carlo Picard sweep", "n": w.n, "queries": w.Q,
                   "samples": w.N, "picard_iterations": w.K, "nu": w.nu, "t": w.t,
                   "draws": "bf16 common table (Philox4x32-10)", "tilt": "Laplace shift from previous iterate",
                   "hamiltonian": w.ham, "coefficient": "min{0,H} (tube equation)" if w.tube else "H",
                   "datum": w.datum},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12, "unit": "TOP/s",
                     "frac": achieved / VALU_PEAK, "traffic": measured_traffic(),
                     "kernel": "pair loop (sweep_pairs_kernel<48, 15>)", "kernel_ms_per_launch": per_launch_ms,
                     "launches_timed": launches, "alu_slots_per_pair": slots},
        "cpu_baseline": cpu,
        # the paper reports CPU timings only: ~2.0e7 query.samples.iterations/s
        # on one core (derived from its 3D Dubins and rocket slice timings)
        "paper_context": {"value": 2.0e7, "unit": "query·samples/s (K iterations counted)",
                          "hardware": "1 core of an Intel Core i7-14700K, JAX CPU backend",
                          "workload": "3D pursuit-evasion slices: 1,600 states, N = 14,000-20,000, K = 12-15",
                          "note": "context only: different workload, machine and precision"},
        "estimator_health": health,
        "surrogate": study,
        "surrogate_exact_case": study_exact,
        "batched": bstudy,
        "flock": fstudy,
        "pursuit_game": pstudy,
        "small_configs": sstudy,
        "time_marching": tstudy,
        "reach_avoid": rastudy,
        "topology": topo,
        "rockets_game": rstudy,
        "murmuration": mstudy,
        "double_integrator": dstudy,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
