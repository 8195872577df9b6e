"""Test helpers: the same problem described to the oracle and to the library,
and the parity tolerances."""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24          # float32 unit roundoff


def oracle_problem(fields: dict, aux=None):
    from oracle import model
    f = dict(fields)
    return model.Problem(datum_aux=aux, **f)


def gpu_problem(fields: dict, aux=None, problem_id: int = 0):
    from paper_2605_18566_amd import ProblemSpec
    return ProblemSpec(datum_aux=aux, problem_id=problem_id, **fields)


def to_dev(a: np.ndarray, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)


def soa(x: np.ndarray) -> np.ndarray:
    """[Q, n] -> [n, Q] float32."""
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32).T)


def value_tol(v_or, c, theta, sigma, lmax):
    """Value tolerance: 1e-4 |v| plus a float32 rounding floor.

    The device forms the log-weight a = -c l(y) - |theta|^2/(2 sigma^2)
    - <z, theta>/sigma in float32; each term carries a relative rounding of a
    few u32, so |delta a| <~ k u32 |c| L with
    L = max|l(y)| + |theta|^2/(2 sigma^2 |c|) + |theta| |z|max/(sigma |c|),
    and v = -(1/c) log mean e^a moves by |delta a|/|c| <= k u32 L.  The sums
    S are float32 within one 128-sample LDS round (relative error <= 128 u32)
    and float64 across rounds, giving another 128 u32/|c|.  k = 64 covers the
    number of roundings on the path with margin.
    """
    c = np.abs(np.asarray(c, dtype=np.float64))
    th2 = np.sum(np.asarray(theta, dtype=np.float64) ** 2, axis=-1) if theta is not None else 0.0
    L = lmax + th2 / (2 * sigma ** 2 * c) + np.sqrt(th2) * 6.0 / (sigma * c)
    return 1e-4 * np.abs(v_or) + 64 * U32 * (1.0 + L) + 128 * U32 / c


def grad_tol(g_or, c, sigma, N):
    """Gradient tolerance: 1e-3 max(|Dv|, 1/(|c| sigma sqrt(N))) per query (2-norm)."""
    gn = np.linalg.norm(g_or, axis=-1)
    return 1e-3 * np.maximum(gn, 1.0 / (np.abs(c) * sigma * np.sqrt(N)))


ESS_RTOL_CAP = 0.5


def ess_rtol(c, theta, sigma, lmax):
    """Relative ESS tolerance.  The log-weight a = -c l - |theta|^2/(2 sigma^2)
    - <z, theta>/sigma is formed in float32 from float32 terms through at most
    16 roundings, so |delta a| <= 16 u32 |c| L with L as in value_tol; that
    moves S by at most that fraction and S2 by twice it, so ESS = S^2/S2 by at
    most four times: 1e-3 + 64 u32 |c| L.  Where this exceeds ESS_RTOL_CAP the
    ESS is not resolved by float32 log-weights at all (|c| L of 1e5 and more:
    the shifted rocket game); those states are excluded from the ESS check
    (their v and Dv keep their tolerances) and counted by the caller.
    Measured on the parity cases: |delta ESS|/ESS <= 20 u32 |c| L."""
    c = np.abs(np.asarray(c, dtype=np.float64))
    th2 = np.sum(np.asarray(theta, dtype=np.float64) ** 2, axis=-1) if theta is not None else 0.0
    cL = c * lmax + th2 / (2 * sigma ** 2) + np.sqrt(th2) * 6.0 / sigma
    return 1e-3 + 64 * U32 * cL
