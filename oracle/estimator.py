"""Monte-Carlo heat-kernel estimators and the Picard loop (CPU oracle, FP64).

TEST INFRASTRUCTURE ONLY.  A plain, slow, direct transcription of the method
for checking the device path; nothing in the product path imports it.

Estimators (appendix: log-sum-exp corollary, Monte-Carlo gradient corollary,
tilted-proposal corollary).  For one query x with frozen coefficient c, shift
theta and sigma^2 = delta t, draws z_i ~ N(0, I):

    y_i = x + theta + sigma z_i
    a_i = -c l(y_i) - |theta|^2 / (2 sigma^2) - <z_i, theta> / sigma
          (log of the tilted weight w_theta(y_i) exp(-c l(y_i)))
    v   = -(1/c) log( (1/N) sum_i exp(a_i) )
    Dv  = (1/(t delta c)) (x - sum_i y_i e^{a_i} / sum_i e^{a_i})
        = -(theta + sigma * Gbar) / (c sigma^2),  Gbar = sum_i e^{a_i} z_i / sum_i e^{a_i}
    ESS = (sum_i e^{a_i})^2 / sum_i e^{2 a_i}   (Section 2.4)

With the control variate option the weighted mean Gbar is replaced by
Gbar - (1/N) sum_i z_i, whose subtracted term has mean zero.

The maximum m = max_i a_i is factored out before exponentiating; this is the
log-sum-exp identity and changes nothing mathematically.

Picard loop: Algorithm 1 -- v^(0) = l, p^(0) = D l, then for k = 0, 1, ...
freeze c^(k) = coefficient(x, p^(k)), estimate v^(k+1), Dv^(k+1), set
p^(k+1) = Dv^(k+1), and stop once ||v^(k+1) - v^(k)|| / ||v^(k)|| < tol
(relative L2 over the evaluation states, as in the caption of Table 2).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np

from . import model, philox


@dataclass
class Estimate:
    v: np.ndarray        # [Q]
    grad: np.ndarray     # [Q, n]
    ess: np.ndarray      # [Q]
    m: np.ndarray        # [Q]  max log-weight
    S: np.ndarray        # [Q]  sum exp(a - m)
    S2: np.ndarray       # [Q]  sum exp(2 (a - m))
    G: np.ndarray        # [Q, n] sum exp(a - m) z
    zbar: np.ndarray     # [Q, n] (1/N) sum z
    lmax: np.ndarray     # [Q]  max |l(y_i)| (scale for rounding floors)


def draws_for(pb: model.Problem, queries: np.ndarray, time_step: int, iteration: int, N: int):
    """z for a chunk of queries: [n, N] (shared table) or [Qc, n, N] (fresh)."""
    if pb.sample_mode == "crn_step":
        return philox.crn_table(pb.seed, pb.problem_id, time_step, pb.n, N, pb.sample_bf16)
    if pb.sample_mode == "fresh":
        return philox.fresh_draws(pb.seed, pb.problem_id, time_step, iteration, queries, pb.n, N,
                                  pb.sample_bf16)
    raise ValueError(pb.sample_mode)


def value_grad(pb: model.Problem, x: np.ndarray, t: float, N: int, c: np.ndarray,
               theta: Optional[np.ndarray] = None, time_step: int = 0, iteration: int = 0,
               z: Optional[np.ndarray] = None, chunk_bytes: float = 2 ** 27,
               datum_fn: Optional[Callable[[np.ndarray], np.ndarray]] = None) -> Estimate:
    """One frozen-coefficient sweep at all queries x[Q, n] (the estimators above).

    z, if given, overrides the generator: shape [n, N] (shared) or [Q, n, N].
    datum_fn, if given, replaces the terminal datum: y [Qc, N, n] -> l [Qc, N].
    """
    x = np.asarray(x, dtype=np.float64)
    Q, n = x.shape
    c = np.asarray(c, dtype=np.float64)
    theta = np.zeros_like(x) if theta is None else np.asarray(theta, dtype=np.float64)
    sigma = np.sqrt(pb.delta * t)
    out = Estimate(np.zeros(Q), np.zeros((Q, n)), np.zeros(Q), np.zeros(Q), np.zeros(Q),
                   np.zeros(Q), np.zeros((Q, n)), np.zeros((Q, n)), np.zeros(Q))
    qc = max(1, int(chunk_bytes // (8 * max(n, 3) * N)))
    shared = None
    if z is None and pb.sample_mode == "crn_step":
        shared = draws_for(pb, None, time_step, 0, N)
    for q0 in range(0, Q, qc):
        qs = np.arange(q0, min(Q, q0 + qc))
        if z is not None:
            zc = z if z.ndim == 2 else z[qs]
        elif shared is not None:
            zc = shared
        else:
            zc = draws_for(pb, qs, time_step, iteration, N)
        zc = np.broadcast_to(zc, (len(qs), n, N)) if zc.ndim == 2 else zc
        zt = np.transpose(zc, (0, 2, 1))                               # [Qc, N, n]
        th = theta[qs]
        y = x[qs, None, :] + th[:, None, :] + sigma * zt               # [Qc, N, n]
        if datum_fn is None:
            aux = None if pb.datum != "knn_balls" else np.asarray(pb.datum_aux)[qs]
            ell = model.datum(pb, y, aux)                              # [Qc, N]
        else:
            ell = np.asarray(datum_fn(y), dtype=np.float64)
        a = (-c[qs, None] * ell
             - np.sum(th * th, axis=1)[:, None] / (2.0 * sigma ** 2)
             - np.einsum("qin,qn->qi", zt, th) / sigma)
        m = np.max(a, axis=1)
        w = np.exp(a - m[:, None])
        S = np.sum(w, axis=1)
        S2 = np.sum(w * w, axis=1)
        G = np.einsum("qi,qin->qn", w, zt)
        zbar = np.mean(zt, axis=1)
        v = -(m + np.log(S / N)) / c[qs]
        gbar = G / S[:, None]
        if pb.grad_cv:
            gbar = gbar - zbar
        grad = -(th + sigma * gbar) / (c[qs, None] * sigma ** 2)
        out.v[qs], out.grad[qs], out.ess[qs] = v, grad, S * S / S2
        out.m[qs], out.S[qs], out.S2[qs], out.G[qs], out.zbar[qs] = m, S, S2, G, zbar
        out.lmax[qs] = np.max(np.abs(ell), axis=1)
    return out


@dataclass
class PicardResult:
    v: np.ndarray
    grad: np.ndarray
    c: np.ndarray            # coefficient frozen in the last executed iteration
    ess: np.ndarray
    flags: np.ndarray        # per-query relative change not <= tol at the last iteration
                             # (a NaN change is flagged), or a non-finite v or gradient
    resid_hist: np.ndarray   # global relative L2 change per executed iteration
    iters_done: int
    lmax: np.ndarray
    theta: np.ndarray        # shift used in the last executed iteration
    rq: np.ndarray           # per-query relative change of the last executed iteration


def v_floor(pb: model.Problem, t: float) -> float:
    """Floor of the per-query relative change denominator: 1e-2 sigma sqrt(n)."""
    return 1e-2 * np.sqrt(pb.delta * t) * np.sqrt(pb.n)


def picard(pb: model.Problem, x: np.ndarray, t: float, N: int, K: int, tol: float = 0.0,
           time_step: int = 0, p0: Optional[np.ndarray] = None, v0: Optional[np.ndarray] = None) -> PicardResult:
    """Algorithm 1 at the evaluation states x[Q, n] and horizon t.

    The "Fix" step starts the loop from v^(0) = l(x) and p^(0) = D l(x); a warm
    start replaces either by the given v0[Q] or p0[Q, n] (the first relative
    change, and so the first residual and flags, is measured from v0).
    """
    x = np.asarray(x, dtype=np.float64)
    Q, n = x.shape
    sigma = np.sqrt(pb.delta * t)
    v_prev = datum_at(pb, x) if v0 is None else np.asarray(v0, dtype=np.float64).copy()
    p = model.datum_grad(pb, x, pb.datum_aux) if p0 is None else np.asarray(p0, dtype=np.float64)
    hist = []
    est = None
    c = theta = None
    rq = np.zeros(Q)
    for k in range(K):
        c = model.coefficient(pb, x, p)
        theta = model.tilt(pb, sigma, c, p)
        est = value_grad(pb, x, t, N, c, theta, time_step=time_step, iteration=k)
        dv = est.v - v_prev
        den = np.sqrt(np.sum(v_prev ** 2))
        r = np.sqrt(np.sum(dv ** 2)) / den if den > 0 else np.sqrt(np.sum(dv ** 2))
        hist.append(r)
        rq = np.abs(dv) / np.maximum(np.abs(v_prev), v_floor(pb, t))
        v_prev = est.v
        p = est.grad
        if r < tol:
            break
    return PicardResult(est.v, est.grad, c, est.ess, _flags(rq, tol, est), np.array(hist), len(hist), est.lmax,
                        theta, rq)


def _flags(rq: np.ndarray, tol: float, est: Estimate) -> np.ndarray:
    """Not converged: the relative change is not within tol (NaN included) or
    the estimate itself is not finite."""
    return ~(rq <= tol) | ~np.isfinite(est.v) | ~np.all(np.isfinite(est.grad), axis=1)


def datum_at(pb: model.Problem, x: np.ndarray) -> np.ndarray:
    """l at the evaluation states themselves (v^(0) = g in Algorithm 1)."""
    aux = np.asarray(pb.datum_aux) if pb.datum == "knn_balls" else None
    return model.datum(pb, np.asarray(x, dtype=np.float64)[:, None, :], aux)[:, 0]


def tube_step(pb: model.Problem, x: np.ndarray, t_prev: float, dt: float, N: int, K: int,
              datum_fn: Callable[[np.ndarray], np.ndarray], v0: np.ndarray, p0: np.ndarray,
              tol: float = 0.0, time_step: int = 0, z: Optional[np.ndarray] = None) -> PicardResult:
    """One step of time marching in semigroup form.

    The value at t_prev + dt solves the same viscous equation over [t_prev,
    t_prev + dt] with v(t_prev, .) as its initial datum (the solution operator
    of the equation is a semigroup; Algorithm 1 needs only a datum and a
    horizon).  So this is Algorithm 1 with the horizon dt (sigma^2 = delta dt),
    the datum y -> v(t_prev, y) given by datum_fn, and the Picard loop started
    from the previous value and its gradient at the states: v^(0) = v0,
    p^(0) = p0 (the "Fix" step of Algorithm 1 with v(t_prev, .) in place of l).
    With the tube flag of the problem the coefficient is frozen from
    min{0, H}, as in the tube equation.  z, if given, overrides the draws as
    in value_grad.
    """
    x = np.asarray(x, dtype=np.float64)
    Q, n = x.shape
    sigma = np.sqrt(pb.delta * dt)
    v_prev = np.asarray(v0, dtype=np.float64).copy()
    p = np.asarray(p0, dtype=np.float64).copy()
    hist = []
    est = None
    c = theta = None
    rq = np.zeros(Q)
    for k in range(K):
        c = model.coefficient(pb, x, p)
        theta = model.tilt(pb, sigma, c, p)
        est = value_grad(pb, x, dt, N, c, theta, time_step=time_step, iteration=k, z=z, datum_fn=datum_fn)
        dv = est.v - v_prev
        den = np.sqrt(np.sum(v_prev ** 2))
        r = np.sqrt(np.sum(dv ** 2)) / den if den > 0 else np.sqrt(np.sum(dv ** 2))
        hist.append(r)
        rq = np.abs(dv) / np.maximum(np.abs(v_prev), v_floor(pb, dt))
        v_prev = est.v
        p = est.grad
        if r < tol:
            break
    return PicardResult(est.v, est.grad, c, est.ess, _flags(rq, tol, est), np.array(hist), len(hist), est.lmax,
                        theta, rq)
