"""Problem data for the CPU oracle: terminal data, Hamiltonians, frozen coefficient, tilt.

TEST INFRASTRUCTURE ONLY (FP64, numpy).  Not imported by the product path.

Conventions (paper, Section 2 and the sign convention under Algorithm 1):
the viscous problem is v_t + H(t; x, Dv) = (delta/2) Lap v with datum
v(0; x) = l(x), t is time-to-go, H = max_u min_w <p, f>.  The datum l is a
signed distance: negative inside the target set.  In terms of the viscosity nu
used by the public interface, delta = 2 nu.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

HAMILTONIANS = ("quadratic", "dubins_pairs", "zero", "double_integrator", "pursuit_evasion", "rockets",
                "murmuration")
DATUMS = ("half_sqnorm", "ball", "min_pair_disks", "knn_balls", "linear", "capture", "disc_union")


@dataclass
class Problem:
    """One problem instance; mirrors the fields of the library's problem record.

    ham_p:   rockets: (a, g, u_max).  murmuration: (v_e, v_p, w_e, w_p,
             g_lo, g_hi).  quadratic/zero: unused.  dubins_pairs: (s, v_e, v_p, w) with s the
             sign of the p2 term (+1 from the relative dynamics, -1 for the form
             the paper prints).  double_integrator: (u_max, s) for n = 2k,
             k = 1..3 (positions, then velocities): s < 0 the control
             minimises H (the paper's time-optimal plant), else it maximises.
             pursuit_evasion: (a_evader, a_pursuer, u_max) for m = n/3 planar
             agents (x, y, heading), the last one the evader.
    datum_p: ball: (k, r) -> ||y[:k]|| - r.  half_sqnorm: unused.
             min_pair_disks: (r,).  knn_balls: (r, K).  linear: (b,).
             capture: (r,) -> min over pursuers of the distance to the evader, - r.
    datum_aux: linear: a[n].  knn_balls: neighbour positions [Q, K, 3].
             disc_union: the K planar centres [K, 2] (datum_p = (r, K)).
    """
    n: int
    ham: str
    datum: str
    nu: float
    ham_p: tuple = (1.0, 1.0, 1.0, 1.0)
    datum_p: tuple = ()
    datum_aux: Optional[np.ndarray] = None
    eta: float = 1e-2
    c_min: float = 1e-2
    c_max: float = 1e4
    tilt: bool = False
    sample_mode: str = "crn_step"      # "fresh" | "crn_step"
    sample_bf16: bool = False
    grad_cv: bool = False
    seed: int = 0
    problem_id: int = 0
    tube: bool = False        # coefficient from min{0, H} (tube equation HJI-RCBRT-Visc)

    @property
    def delta(self) -> float:
        return 2.0 * self.nu


# --------------------------------------------------------------------------- datum
def datum(pb: Problem, y: np.ndarray, q_aux: Optional[np.ndarray] = None) -> np.ndarray:
    """l(y) for y[..., n].

    q_aux is the per-query auxiliary data of knn_balls: [K, 3] for one query,
    or [Qc, K, 3] when y has shape [Qc, N, n].
    """
    kind = pb.datum
    if kind == "half_sqnorm":
        return 0.5 * np.sum(y * y, axis=-1)
    if kind == "ball":
        k, r = int(pb.datum_p[0]), float(pb.datum_p[1])
        return np.sqrt(np.sum(y[..., :k] ** 2, axis=-1)) - r
    if kind == "min_pair_disks":
        r = float(pb.datum_p[0])
        m = pb.n // 3
        rho2 = y[..., 0:3 * m:3] ** 2 + y[..., 1:3 * m:3] ** 2
        return np.sqrt(np.min(rho2, axis=-1)) - r
    if kind == "knn_balls":
        r = float(pb.datum_p[0])
        nb = np.asarray(q_aux, dtype=np.float64)           # [K, 3] or [Qc, K, 3]
        if nb.ndim == 3:                                   # y is [Qc, N, n]
            nb = nb[:, None, :, :]
        d2 = np.sum((y[..., None, :3] - nb) ** 2, axis=-1)  # [..., K]
        return np.sqrt(np.min(d2, axis=-1)) - r
    if kind == "linear":
        a = np.asarray(pb.datum_aux, dtype=np.float64)
        return y @ a + float(pb.datum_p[0])
    if kind == "capture":
        # target set of the multi-pursuer game (Section 3.2): some pursuer within
        # r of the evader, the evader being the last agent
        r = float(pb.datum_p[0])
        m = pb.n // 3
        e = 3 * (m - 1)
        d2 = (y[..., 0:e:3] - y[..., e:e + 1]) ** 2 + (y[..., 1:e:3] - y[..., e + 1:e + 2]) ** 2
        return np.sqrt(np.min(d2, axis=-1)) - r
    if kind == "disc_union":
        # union of capture cylinders about fixed planar centres (appendix,
        # murmuration setup): min_j |(y0, y1) - c_j| - r
        r = float(pb.datum_p[0])
        cen = np.asarray(pb.datum_aux, dtype=np.float64).reshape(-1, 2)
        d2 = (y[..., 0:1] - cen[:, 0]) ** 2 + (y[..., 1:2] - cen[:, 1]) ** 2
        return np.sqrt(np.min(d2, axis=-1)) - r
    raise ValueError(f"unknown datum {kind}")


def datum_grad(pb: Problem, x: np.ndarray, aux_all: Optional[np.ndarray] = None) -> np.ndarray:
    """Analytic D l(x) for x[Q, n] (Algorithm 1 initialises the coefficient from Dg).

    At a kink the rule is: radius 0 gives 0; ties in a minimum go to the
    lowest index.
    """
    Q, n = x.shape
    g = np.zeros_like(x)
    kind = pb.datum
    if kind == "half_sqnorm":
        return x.copy()
    if kind == "ball":
        k = int(pb.datum_p[0])
        rho = np.sqrt(np.sum(x[:, :k] ** 2, axis=1))
        safe = np.where(rho > 0, rho, 1.0)
        g[:, :k] = np.where(rho[:, None] > 0, x[:, :k] / safe[:, None], 0.0)
        return g
    if kind == "min_pair_disks":
        m = n // 3
        rho2 = x[:, 0:3 * m:3] ** 2 + x[:, 1:3 * m:3] ** 2
        j = np.argmin(rho2, axis=1)                       # first minimum
        rho = np.sqrt(rho2[np.arange(Q), j])
        safe = np.where(rho > 0, rho, 1.0)
        for d in (0, 1):
            col = 3 * j + d
            g[np.arange(Q), col] = np.where(rho > 0, x[np.arange(Q), col] / safe, 0.0)
        return g
    if kind == "knn_balls":
        nb = np.asarray(aux_all, dtype=np.float64)        # [Q, K, 3]
        diff = x[:, None, :3] - nb
        d2 = np.sum(diff ** 2, axis=-1)
        j = np.argmin(d2, axis=1)
        dj = diff[np.arange(Q), j]
        dist = np.sqrt(d2[np.arange(Q), j])
        safe = np.where(dist > 0, dist, 1.0)
        g[:, :3] = np.where(dist[:, None] > 0, dj / safe[:, None], 0.0)
        return g
    if kind == "linear":
        return np.broadcast_to(np.asarray(pb.datum_aux, dtype=np.float64), x.shape).copy()
    if kind == "capture":
        m = n // 3
        e = 3 * (m - 1)
        dx = x[:, 0:e:3] - x[:, e:e + 1]
        dy = x[:, 1:e:3] - x[:, e + 1:e + 2]
        d2 = dx * dx + dy * dy
        j = np.argmin(d2, axis=1)                          # first minimum
        rho = np.sqrt(d2[np.arange(Q), j])
        safe = np.where(rho > 0, rho, 1.0)
        gx = np.where(rho > 0, dx[np.arange(Q), j] / safe, 0.0)
        gy = np.where(rho > 0, dy[np.arange(Q), j] / safe, 0.0)
        g[np.arange(Q), 3 * j] = gx
        g[np.arange(Q), 3 * j + 1] = gy
        g[:, e] = -gx
        g[:, e + 1] = -gy
        return g
    if kind == "disc_union":
        cen = np.asarray(pb.datum_aux, dtype=np.float64).reshape(-1, 2)
        dx = x[:, 0:1] - cen[:, 0]
        dy = x[:, 1:2] - cen[:, 1]
        d2 = dx * dx + dy * dy
        j = np.argmin(d2, axis=1)                          # first minimum
        rho = np.sqrt(d2[np.arange(Q), j])
        safe = np.where(rho > 0, rho, 1.0)
        g[:, 0] = np.where(rho > 0, dx[np.arange(Q), j] / safe, 0.0)
        g[:, 1] = np.where(rho > 0, dy[np.arange(Q), j] / safe, 0.0)
        return g
    raise ValueError(f"unknown datum {kind}")


# ----------------------------------------------------------------------- Hamiltonian
def hamiltonian(pb: Problem, x: np.ndarray, p: np.ndarray) -> np.ndarray:
    """H(x, p) = max_u min_w <p, f(x, u, w)> for x, p of shape [Q, n]."""
    kind = pb.ham
    if kind == "quadratic":
        return 0.5 * np.sum(p * p, axis=1)
    if kind == "zero":
        return np.zeros(x.shape[0])
    if kind == "dubins_pairs":
        # Relative Dubins dynamics (appendix, Dubins pursuit-evasion):
        # x1' = -v_e + v_p cos x3 + w_e x2, x2' = v_p sin x3 - w_e x1, x3' = w_p - w_e;
        # the evader turn rate w_e in [-w, w] maximises, the pursuer's w_p minimises.
        s, ve, vp, w = (float(v) for v in pb.ham_p[:4])
        m = pb.n // 3
        H = np.zeros(x.shape[0])
        for j in range(m):
            x1, x2, x3 = x[:, 3 * j], x[:, 3 * j + 1], x[:, 3 * j + 2]
            p1, p2, p3 = p[:, 3 * j], p[:, 3 * j + 1], p[:, 3 * j + 2]
            H += (p1 * (vp * np.cos(x3) - ve) + s * p2 * vp * np.sin(x3)
                  + w * np.abs(p1 * x2 - p2 * x1 - p3) - w * np.abs(p3))
        return H
    if kind == "pursuit_evasion":
        # m planar agents (Section 3.2): x_i' = a_i cos th_i, y_i' = a_i sin th_i,
        # th_i' = u_i with |u_i| <= u_max; the evader (last agent) maximises, the
        # pursuers minimise, so the turn terms give +u_max|p_th| and -u_max|p_th|.
        ae, ap, umax = (float(v) for v in pb.ham_p[:3])
        m = pb.n // 3
        H = np.zeros(x.shape[0])
        for j in range(m):
            a = ae if j == m - 1 else ap
            th = x[:, 3 * j + 2]
            H += a * (p[:, 3 * j] * np.cos(th) + p[:, 3 * j + 1] * np.sin(th))
            H += (umax if j == m - 1 else -umax) * np.abs(p[:, 3 * j + 2])
        return H
    if kind == "rockets":
        # Two rockets on a plane (appendix, game of two rockets), relative
        # state (x, z, theta): with the rows of the Hamiltonian's definition,
        # x' = a cos th + u_e x, z' = a sin th + a + u_p x - g, th' = u_p - u_e,
        # and H = -max_{u_e} min_{u_p} <p, f> over |u| <= u_max.
        a, g, umax = (float(v) for v in pb.ham_p[:3])
        xx, th = x[:, 0], x[:, 2]
        p1, p2, p3 = p[:, 0], p[:, 1], p[:, 2]
        inner = a * p1 * np.cos(th) + p2 * (a + a * np.sin(th) - g)
        return -(inner + umax * np.abs(p1 * xx - p3) - umax * np.abs(p2 * xx + p3))
    if kind == "murmuration":
        # the individual under attack in a flock (appendix, murmuration
        # Hamiltonian), relative state (x1, x2, altitude x3, heading x4), as
        # printed in its general form:
        # p1 (v_e - v_p cos x4) - p2 v_p sin x4 - w_p |p4|
        #   + w_e |p2 x1 - p1 x2 + p4| + g_lo |p3| - g_hi |p3|
        ve, vp, we, wp, glo, ghi = (float(v) for v in pb.ham_p[:6])
        x1, x2, x4 = x[:, 0], x[:, 1], x[:, 3]
        p1, p2, p3, p4 = p[:, 0], p[:, 1], p[:, 2], p[:, 3]
        return (p1 * (ve - vp * np.cos(x4)) - p2 * vp * np.sin(x4) - wp * np.abs(p4)
                + we * np.abs(p2 * x1 - p1 * x2 + p4) + glo * np.abs(p3) - ghi * np.abs(p3))
    if kind == "double_integrator":
        # pos' = vel, vel' = u with ||u|| <= u_max (k = n/2 axes): the control
        # maximises <p, f> (+u_max ||p_vel||) or, with ham_p[1] < 0, minimises it
        # (-u_max ||p_vel||; the double integral plant of the appendix, where
        # u = -sign(p2) gives H = p1 x2 - |p2|)
        k = pb.n // 2
        umax = float(pb.ham_p[0])
        s = -1.0 if len(pb.ham_p) > 1 and float(pb.ham_p[1]) < 0 else 1.0
        return (np.sum(p[:, :k] * x[:, k:2 * k], axis=1)
                + s * umax * np.sqrt(np.sum(p[:, k:2 * k] ** 2, axis=1)))
    raise ValueError(f"unknown Hamiltonian {kind}")


def coefficient(pb: Problem, x: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Frozen coefficient c = (2/delta) H / (|p|^2 + eta), sign kept, |c| clipped.

    Follows the coefficient definition of Section 2.1, its regularised form
    (lemma on the regularised coefficient) and the clipping of |c| to
    [c_min, c_max] with the sign kept (remark on the sign of the coefficient);
    sign(0) is taken as +1.  For H = |p|^2/2 the exact constant 1/delta is used
    with no regularisation (exact Cole-Hopf case).  For the tube equation
    (HJI-RCBRT-Visc, v_t + min{0, H} = (delta/2) Lap v) H is replaced by
    min{0, H}.
    """
    if pb.ham == "quadratic":
        return np.full(x.shape[0], 1.0 / pb.delta)
    H = hamiltonian(pb, x, p)
    if pb.tube:
        H = np.minimum(H, 0.0)
    return frozen_coefficient(H, p, pb.delta, pb.eta, pb.c_min, pb.c_max)


def frozen_coefficient(H: np.ndarray, p: np.ndarray, delta: float, eta: float, c_min: float,
                       c_max: float) -> np.ndarray:
    """The general branch of the coefficient from Hamiltonian values H[Q] and p[Q, n].

    c_raw = (2/delta) H / (|p|^2 + eta) (the coefficient definition with the
    regularised denominator), then |c| clipped to [c_min, c_max] with the sign
    of c_raw kept and sign(0) = +1 (remark on the sign of the coefficient).
    """
    c_raw = (2.0 / delta) * np.asarray(H, dtype=np.float64) / (np.sum(p * p, axis=1) + eta)
    sgn = np.where(c_raw < 0, -1.0, 1.0)
    return sgn * np.clip(np.abs(c_raw), c_min, c_max)


def tilt(pb: Problem, sigma: float, c: np.ndarray, p: np.ndarray) -> np.ndarray:
    """theta = -sigma^2 c p (first-order Laplace shift of the tilted proposal), or 0."""
    if not pb.tilt:
        return np.zeros_like(p)
    return -(sigma ** 2) * c[:, None] * p
