"""Topology markers of the zero-sublevel set on 2D slices (CPU oracle).  TEST
INFRASTRUCTURE ONLY.

Written from the paper's detection algorithm (appendix on vacuole nucleation
topology): on an m x m slice of v, label the connected components of
{v <= 0} (scipy.ndimage.label, its default 4-connectivity), count as beta_1
the components of the complement {v > 0} that are encircled (touch no edge
of the grid), chi = n_comp - beta_1; between consecutive steps, the event
rules: chi_{t+1} - chi_t < -0.5 -> vacuole nucleation, beta_1(t) >= 1 with
beta_1(t-1) = 0 -> cordon formation, n_comp(t) > n_comp(t-1) -> flock
fragmentation.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

VACUOLE, CORDON, FRAGMENTATION = 1, 2, 4


def markers(v: np.ndarray):
    """(n_comp, beta_1, chi) of one slice v [ny, nx]."""
    inside = np.asarray(v) <= 0
    _, n_comp = ndimage.label(inside)
    lab_out, n_out = ndimage.label(~inside)
    border = np.unique(np.concatenate([lab_out[0], lab_out[-1], lab_out[:, 0], lab_out[:, -1]]))
    border = border[border > 0]
    beta1 = n_out - len(border)
    return int(n_comp), int(beta1), int(n_comp - beta1)


def events(chi, beta1, ncomp):
    """Event bits per step (step 0 has no predecessor)."""
    T = len(chi)
    out = np.zeros(T, dtype=np.int32)
    for t in range(1, T):
        if chi[t] - chi[t - 1] < -0.5:
            out[t] |= VACUOLE
        if beta1[t] >= 1 and beta1[t - 1] == 0:
            out[t] |= CORDON
        if ncomp[t] > ncomp[t - 1]:
            out[t] |= FRAGMENTATION
    return out
