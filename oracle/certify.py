"""Conservative safety certification (CPU oracle, FP64).  TEST INFRASTRUCTURE ONLY.

Written from the paper:
* the total error budget E(K, N, delta, delta_p) = C1 rho^K
  + C2 sqrt(log(1/delta_p) / N) + eps_QL + C3 sqrt(delta) of the total-error
  theorem (remark after it);
* the classification of the conservative-certification corollary: SAFE only
  if v > E, UNSAFE only if v < -E, UNDETERMINED otherwise (a state is unsafe
  iff v <= 0);
* a per-state sampling margin from the finite-sample concentration theorem
  of the frozen-coefficient estimator: with Z = exp(-c g) in [alpha, beta]
  (alpha, beta = the smaller and larger of exp(-c g_min), exp(-c g_max), the
  remark on the sign of the coefficient), mu = E[Z],
      P(|v_hat - v_c| >= eps) <= 2 exp(-2 N mu^2 (1 - exp(-|c| eps))^2 / (beta - alpha)^2),
  so at confidence delta_p: r = (beta - alpha) / mu * sqrt(log(2/delta_p) / (2N)),
  eps = -log(1 - r) / |c| when r < 1, else no finite margin.  The mean mu is
  taken as exp(-c v_hat) (the estimate itself; the paper allows a sharper
  estimate of mu in place of its lower bound alpha), or passed in.
"""
from __future__ import annotations

import numpy as np

SAFE, UNDETERMINED, UNSAFE = 1, 0, -1


def error_budget(C1, rho, K, C2, N, delta_p, eps_ql, C3, delta):
    return C1 * rho ** K + C2 * np.sqrt(np.log(1.0 / delta_p) / N) + eps_ql + C3 * np.sqrt(delta)


def classify(v, E, margin=None):
    """Labels (+1 SAFE, -1 UNSAFE, 0 UNDETERMINED) with margin E (+ per-state margin)."""
    v = np.asarray(v, dtype=np.float64)
    m = E + (0.0 if margin is None else np.asarray(margin, dtype=np.float64))
    out = np.zeros(v.shape, dtype=np.int8)
    out[v > m] = SAFE
    out[v < -m] = UNSAFE
    return out


def mc_margin(v, c, N, delta_p, g_min, g_max=np.inf, mu=None):
    """Per-state sampling margin eps (inf where the bound gives none)."""
    v = np.asarray(v, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        e1, e2 = np.exp(-c * g_min), np.exp(-c * g_max)
        alpha, beta = np.minimum(e1, e2), np.maximum(e1, e2)
        mu = np.exp(-c * v) if mu is None else np.asarray(mu, dtype=np.float64)
        r = (beta - alpha) / mu * np.sqrt(np.log(2.0 / delta_p) / (2.0 * N))
        eps = np.where(r < 1.0, -np.log1p(-np.minimum(r, 1.0)) / np.abs(c), np.inf)
    return eps
