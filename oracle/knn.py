"""Brute-force k nearest neighbours of every agent of a flock (test infrastructure).

The per-agent target set of the flock workload is the union of balls about an
agent's k nearest other agents (topological neighbour rule of the flocking
example; union of signed-distance functions is their minimum).  Distances are
squared Euclidean distances of float32 positions computed in float32 as
(dx*dx + dy*dy) + dz*dz, each operation rounded on its own, so that equal
inputs give the same neighbour decisions on any correctly rounded machine.
Neighbours are ordered by (squared distance, index): ties go to the lower
index.  An agent is never its own neighbour.
"""
from __future__ import annotations

import numpy as np


def dist2_f32(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Squared distances between float32 points a [..., 3] and b [..., 3], in float32."""
    d = (np.asarray(b, np.float32) - np.asarray(a, np.float32)).astype(np.float32)
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def knn(pos: np.ndarray, k: int, queries=None, chunk: int = 512) -> np.ndarray:
    """Indices [Qs, k] of the k nearest other agents of each queried agent.

    pos: [M, 3] float32 agent positions; queries: agent indices (default all).
    """
    pos = np.asarray(pos, np.float32)
    M = pos.shape[0]
    if not 1 <= k < M:
        raise ValueError("need 1 <= k < number of agents")
    qs = np.arange(M) if queries is None else np.asarray(queries)
    out = np.empty((len(qs), k), dtype=np.int64)
    idx = np.arange(M)
    for s in range(0, len(qs), chunk):
        q = qs[s:s + chunk]
        d2 = dist2_f32(pos[q][:, None, :], pos[None, :, :])          # [c, M]
        d2[np.arange(len(q)), q] = np.inf                             # not its own neighbour
        for r in range(len(q)):
            order = np.lexsort((idx, d2[r]))                          # by distance, then index
            out[s + r] = order[:k]
    return out
