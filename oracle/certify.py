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
  estimate of mu in place of its lower bound alpha), or passed in;
* the variance-aware margin the paper's remark on Bernstein bounds points to,
  from the empirical Bernstein inequality (Maurer and Pontil, 2009, Thm. 4,
  two-sided: confidence split between the two tails): with the sample mean
  Zbar, the unbiased sample variance V and the range R = beta - alpha,
      |Zbar - mu| <= sqrt(2 V log(4/delta_p) / N) + 7 R log(4/delta_p) / (3 (N - 1)),
  and V / Zbar^2 = N/(N-1) (N / ESS - 1) in terms of the effective sample
  size ESS = S^2 / S2 of the sweep; with rho = |Zbar - mu| / Zbar < 1 the
  value error is at most -log(1 - rho) / |c|.
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


def bernstein_margin(v, c, ess, N, delta_p, g_min, g_max=np.inf):
    """Per-state margin from the empirical Bernstein inequality (inf where none)."""
    v = np.asarray(v, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    ess = np.asarray(ess, dtype=np.float64)
    L = np.log(4.0 / delta_p)
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        e1, e2 = np.exp(-c * g_min), np.exp(-c * g_max)
        R = np.maximum(e1, e2) - np.minimum(e1, e2)
        zbar = np.exp(-c * v)
        var_rel = N / (N - 1.0) * np.maximum(N / ess - 1.0, 0.0)
        rho = np.sqrt(2.0 * var_rel * L / N) + 7.0 * (R / zbar) * L / (3.0 * (N - 1.0))
        eps = np.where(rho < 1.0, -np.log1p(-np.minimum(rho, 1.0)) / np.abs(c), np.inf)
    return eps
