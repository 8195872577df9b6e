"""Marching-squares isocontours of a 2D slice (CPU oracle).  TEST
INFRASTRUCTURE ONLY.

The zero-level contours the paper draws on its BRT slices (marching squares
on the m x m grid).  Cell (x, y) has corners c0 = (x, y), c1 = (x+1, y),
c2 = (x+1, y+1), c3 = (x, y+1) and edges e0 = c0-c1, e1 = c1-c2, e2 = c2-c3,
e3 = c3-c0.  A corner is inside when v <= level.  An edge with one inside
and one outside corner is crossed at the linear interpolation point
t = (level - v_a) / (v_b - v_a) from its first corner.  A cell with two
crossed edges gives the segment joining them; the two saddle cells (inside
corners c0, c2 or c1, c3) give two segments, decided by the mean of the four
corners (the cell centre): if the centre is inside, the inside corners are
joined through it and the segments cut off the outside corners, else they
cut off the inside corners.  Coordinates are (column, row) grid units.
"""
from __future__ import annotations

import numpy as np

CORNERS = ((0, 0), (1, 0), (1, 1), (0, 1))
EDGES = ((0, 1), (1, 2), (2, 3), (3, 0))
# corner -> the two edges that meet at it
AROUND = {0: (3, 0), 1: (0, 1), 2: (1, 2), 3: (2, 3)}


def _point(x, y, vals, e, level):
    a, b = EDGES[e]
    va, vb = vals[a], vals[b]
    t = (level - va) / (vb - va)
    t = min(max(t, 0.0), 1.0)
    (ax, ay), (bx, by) = CORNERS[a], CORNERS[b]
    return (x + ax + t * (bx - ax), y + ay + t * (by - ay))


def segments(v: np.ndarray, level: float = 0.0) -> np.ndarray:
    """All segments [S, 4] (x0, y0, x1, y1) of one slice v [ny, nx]."""
    v = np.asarray(v, dtype=np.float64)
    ny, nx = v.shape
    out = []
    for y in range(ny - 1):
        for x in range(nx - 1):
            vals = (v[y, x], v[y, x + 1], v[y + 1, x + 1], v[y + 1, x])
            inside = [val <= level for val in vals]
            crossed = [e for e, (a, b) in enumerate(EDGES) if inside[a] != inside[b]]
            if len(crossed) == 2:
                pairs = [tuple(crossed)]
            elif len(crossed) == 4:
                centre_in = np.mean(vals) <= level
                ins = [c for c in range(4) if inside[c]]
                outs = [c for c in range(4) if not inside[c]]
                cut = outs if centre_in else ins
                pairs = [AROUND[c] for c in cut]
            else:
                pairs = []
            for ea, eb in pairs:
                p, q = _point(x, y, vals, ea, level), _point(x, y, vals, eb, level)
                out.append((p[0], p[1], q[0], q[1]))
    return np.array(out, dtype=np.float64).reshape(-1, 4)


def canonical(seg: np.ndarray, decimals: int = 5) -> np.ndarray:
    """Segments with ordered endpoints, rounded, sorted (order-free comparison)."""
    seg = np.asarray(seg, dtype=np.float64).reshape(-1, 4)
    a, b = seg[:, :2], seg[:, 2:]
    swap = (a[:, 0] > b[:, 0]) | ((a[:, 0] == b[:, 0]) & (a[:, 1] > b[:, 1]))
    lo = np.where(swap[:, None], b, a)
    hi = np.where(swap[:, None], a, b)
    s = np.round(np.concatenate([lo, hi], 1), decimals)
    return s[np.lexsort(s.T[::-1])]
