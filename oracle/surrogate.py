"""The surrogate-accelerated sweep, written out step by step (CPU oracle, FP64).

TEST INFRASTRUCTURE ONLY.  Not imported by the product path.

The paper has no learned part; this is the reading of a surrogate that serves
as a Picard warm start, with the plain Monte-Carlo estimator as the judge and
fallback:

  1. the network's outputs at the evaluation states give the warm start
     v^(0) = v_S(x, t) and p^(0) = Dv_S(x, t) (the "Fix" step of Algorithm 1
     with the surrogate in place of the datum), so the first frozen
     coefficient and proposal shift come from the surrogate;
  2. Algorithm 1 runs from there with N_s draws and at most K_s iterations,
     stopping on the relative L2 change tol; a state whose last relative
     change is not within tol (or whose estimate is not finite) is flagged;
  3. each flagged state is solved again by the plain method (v^(0) = l,
     p^(0) = D l) with N_fb draws and K_fb iterations, which replaces its
     result.

Draws come from the common table of (problem, time step), so a state's draws
do not depend on which other states are solved with it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import estimator, mlp, model


@dataclass
class SweepResult:
    v: np.ndarray
    grad: np.ndarray
    fell_back: np.ndarray        # bool [Q]
    warm: estimator.PicardResult
    plain: object                # estimator.PicardResult of the flagged states (in index order), or None
    v_s: np.ndarray              # surrogate outputs at the states
    g_s: np.ndarray


def sweep(pb: model.Problem, params, norm, x: np.ndarray, t: float, N_s: int, K_s: int, N_fb: int, K_fb: int,
          tol: float, time_step: int = 0) -> SweepResult:
    if pb.sample_mode != "crn_step":
        raise ValueError("the surrogate sweep reads a common table")
    x = np.asarray(x, dtype=np.float64)
    v_s, g_s = mlp.value_grad_at(params, norm, x, t)
    warm = estimator.picard(pb, x, t, N_s, K_s, tol=tol, time_step=time_step, p0=g_s, v0=v_s)
    flags = warm.flags
    v, grad = warm.v.copy(), warm.grad.copy()
    idx = np.flatnonzero(flags)
    plain = None
    if idx.size:
        plain = estimator.picard(pb, x[idx], t, N_fb, K_fb, tol=0.0, time_step=time_step)
        v[idx], grad[idx] = plain.v, plain.grad
    return SweepResult(v, grad, flags, warm, plain, v_s, g_s)
