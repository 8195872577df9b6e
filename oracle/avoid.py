"""Reach-avoid tube in splitting form (FP64 oracle).

TEST INFRASTRUCTURE: imported only by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.

The paper states the viscous reach-avoid tube (HJI-RCBRAT-Visc, Section
"Relations to Backward Reachable Sets/Tubes", and the reach-avoid tube of the
appendix) only as a variational inequality whose obstacle term is garbled.
Reading taken here: the avoid set is A = {l_A <= 0} for a level function l_A
(a signed distance, negative inside A), and the value obeys the obstacle
constraint v >= -l_A at every time, so a state of A always has v > 0 and is
never counted as reached.  In splitting form one time step is the ordinary
step (Algorithm 1 over the step's horizon) followed by the projection onto
that constraint, done here.
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np

from . import model


def obstacle_level(pb: model.Problem, x: np.ndarray, aux_all: Optional[np.ndarray] = None
                   ) -> Tuple[np.ndarray, np.ndarray]:
    """l_A(x) and D l_A(x) for x [Q, n]; the datum of pb describes A (kinks and
    ties as the datum rules).  aux_all is the per-state neighbour data of
    knn_balls ([Q, K, 3])."""
    x = np.asarray(x, dtype=np.float64)
    if pb.datum == "knn_balls":
        lv = np.array([model.datum(pb, x[q], q_aux=aux_all[q]) for q in range(x.shape[0])])
    else:
        lv = model.datum(pb, x)
    return np.asarray(lv, dtype=np.float64), model.datum_grad(pb, x, aux_all)


def project(pb: model.Problem, x: np.ndarray, v: np.ndarray, grad: Optional[np.ndarray] = None,
            aux_all: Optional[np.ndarray] = None):
    """Projection onto the obstacle constraint: v <- max(v, -l_A(x)), and where
    the constraint wins (strictly -l_A > v) the gradient becomes -D l_A.

    Returns (v_out, grad_out or None, active)."""
    lv, dl = obstacle_level(pb, x, aux_all)
    h = -lv
    v = np.asarray(v, dtype=np.float64)
    active = h > v
    v_out = np.where(active, h, v)
    g_out = None
    if grad is not None:
        g_out = np.where(active[:, None], -dl, np.asarray(grad, dtype=np.float64))
    return v_out, g_out, active
