"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

Holds workload parameters and query generators only -- none of the method's
arithmetic.  Queries come from numpy's PCG64 stream seeded with
[2605, 18566, config, trial]; the Philox key of a workload is
0x0002605185660000 + 16 config + trial.  All inputs are synthetic with the
shapes, sizes and distributions of the workloads they stand for (the paper
measures on no public dataset).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

PI = math.pi


def rng(cfg: int, trial: int = 0) -> np.random.Generator:
    return np.random.default_rng([2605, 18566, cfg, trial])


def philox_seed(cfg: int, trial: int = 0) -> int:
    return 0x0002605185660000 + 16 * cfg + trial


@dataclass
class Workload:
    """Parameters of one sweep workload (the fields of the problem record plus sizes)."""
    name: str
    n: int
    ham: str
    datum: str
    nu: float
    t: float
    Q: int
    N: int
    K: int
    box: Tuple[Tuple[float, float], ...]
    ham_p: Tuple[float, ...] = (1.0, 1.0, 1.0, 1.0)
    datum_p: Tuple[float, ...] = ()
    eta: float = 1e-2
    c_min: float = 1e-2
    c_max: float = 1e4
    tilt: bool = False
    sample_mode: str = "crn_step"
    sample_bf16: bool = False
    grad_cv: bool = False
    cfg: int = 0
    time_steps: int = 1
    T: float = 1.0
    tube: bool = False

    @property
    def seed(self) -> int:
        return philox_seed(self.cfg)

    def resized(self, **kw) -> "Workload":
        return replace(self, **kw)

    def problem_fields(self) -> dict:
        return dict(n=self.n, ham=self.ham, datum=self.datum, nu=self.nu, ham_p=tuple(self.ham_p),
                    datum_p=tuple(self.datum_p), eta=self.eta, c_min=self.c_min, c_max=self.c_max,
                    tilt=self.tilt, sample_mode=self.sample_mode, sample_bf16=self.sample_bf16,
                    grad_cv=self.grad_cv, seed=self.seed, tube=self.tube)


def queries(w: Workload, Q: Optional[int] = None, trial: int = 0) -> np.ndarray:
    """Uniform queries in the workload's box, float32 [Q, n]."""
    Q = w.Q if Q is None else Q
    g = rng(w.cfg, trial)
    lo = np.array([b[0] for b in w.box])
    hi = np.array([b[1] for b in w.box])
    return (lo + (hi - lo) * g.random((Q, w.n))).astype(np.float32)


def dubins_box(m: int):
    return tuple([(-3.0, 3.0), (-3.0, 3.0), (-PI, PI)] * m)


# Plain MC, n = 2, H = |p|^2/2, nu = 0.05, t = 0.5, disk SDF; 4,096 queries in
# [-2, 2]^2, N = 8,192 draws per query, one Picard iteration.
C1 = Workload("c1_quadratic_disk_n2", n=2, ham="quadratic", datum="ball", datum_p=(2, 1.0), nu=0.05, t=0.5,
              Q=4096, N=8192, K=1, box=((-2.0, 2.0), (-2.0, 2.0)), sample_mode="fresh", cfg=1)
C1_QUAD = replace(C1, name="c1_quadratic_halfsq_n2", datum="half_sqnorm", datum_p=())

# Dubins pursuit-evasion in relative coordinates, disk of radius 0.5, nu = 0.01,
# T = 1 in 10 horizons, 5 iterations, 65,536 queries, N = 65,536 common draws.
# The Dubins game is a reachability (tube) problem: its coefficient uses
# min{0, H} (tube equation of the paper's Dubins example).
C2 = Workload("c2_dubins_n3", n=3, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=0.01, t=1.0,
              Q=65536, N=65536, K=5, box=dubins_box(1), tilt=True, sample_mode="crn_step", cfg=2,
              time_steps=10, T=1.0, tube=True)

# n = 45: 15 stacked relative Dubins pairs, nu = 0.01, T = 1, bfloat16 common
# draws, N = 65,536, K = 5, 262,144 queries (the surrogate's inference size).
C5 = Workload("c5_dubins15_n45", n=45, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=0.01,
              t=1.0, Q=262144, N=65536, K=5, box=dubins_box(15), tilt=True, sample_mode="crn_step",
              sample_bf16=True, cfg=5, tube=True)

# The same n = 45 datum, draws and sizes with H = |p|^2/2, the exact Cole-Hopf
# case (no quasi-linearisation defect): the workload of the equal-accuracy
# surrogate study.
C5Q = replace(C5, name="c5q_quadratic15_n45", ham="quadratic", tube=False, cfg=6)


# Flock safety: 100,000 agents with 6D states (position uniform in [0, 50]^3,
# velocity N(0, 0.5^2 I)); an agent's target set is the union of balls of
# radius 0.2 about its 7 nearest other agents (hash grid with cell 2);
# double-integrator H with |u| <= 1, tube coefficient, nu = 0.02, T = 1 in 5
# horizons, 3 iterations, N = 4,096 bfloat16 common draws, Laplace shift.
C4 = Workload("c4_flock_n6", n=6, ham="double_integrator", ham_p=(1.0,), datum="knn_balls", datum_p=(0.2, 7),
              nu=0.02, t=1.0, Q=100000, N=4096, K=3, box=((0.0, 50.0),) * 3 + ((-1.5, 1.5),) * 3, tilt=True,
              sample_mode="crn_step", sample_bf16=True, cfg=4, time_steps=5, T=1.0, tube=True)
FLOCK_EXTENT, FLOCK_CELL, FLOCK_VEL_STD = 50.0, 2.0, 0.5


def flock_agents(M: int = 100000, trial: int = 0, extent: Optional[float] = None) -> np.ndarray:
    """Agent states [M, 6] float32: positions uniform in [0, extent]^3 (default:
    the 100,000-agent density, extent 50 (M / 1e5)^(1/3)), velocities N(0, 0.5^2 I)."""
    if extent is None:
        extent = FLOCK_EXTENT * (M / 100000) ** (1.0 / 3.0)
    g = rng(4, trial)
    pos = g.uniform(0.0, extent, (M, 3))
    vel = g.normal(0.0, FLOCK_VEL_STD, (M, 3))
    return np.concatenate([pos, vel], 1).astype(np.float32)


# The paper's 45-dimensional multi-pursuer single-evader game (Section 3.2,
# Table 2): 14 pursuers and one evader (the last agent), capture radius 1.5,
# three speed regimes; delta = 0.08 (nu = 0.04) as in the paper's 3D games,
# N = 20,000 draws (the 7.2 MB per iteration the paper reports at n = 45),
# K = 15 iterations, 1,600 evaluation states (a 40 x 40 slice's count) with
# positions uniform over [-100, 100] per coordinate (the paper's statement for
# this game) and headings in [-pi, pi), t = 1.
def pursuit_box(m: int, half: float = 100.0):
    return tuple([(-half, half), (-half, half), (-PI, PI)] * m)


PURSUIT_REGIMES = {"evader_faster": (2.0, 1.0), "equal_speed": (1.0, 1.0), "pursuers_faster": (1.0, 2.0)}
# The plain estimator (no shift): with the Laplace shift the importance
# weights of this game degenerate (median ESS ~ 3 of 4,096) and the iteration
# does not contract; without it the median ESS is ~ 1,400.
C6 = Workload("c6_pursuit15_n45", n=45, ham="pursuit_evasion", ham_p=(2.0, 1.0, 1.0), datum="capture",
              datum_p=(1.5,), nu=0.04, t=1.0, Q=1600, N=20000, K=15, box=pursuit_box(15), tilt=False,
              sample_mode="crn_step", sample_bf16=True, cfg=7, tube=True)


# The paper's two-rocket game (appendix, game of two rockets; Table 1):
# relative state (x, z, theta), a = 64, g = 32 (ft/s^2), |u| <= 1, capture
# radius 1.5 in (x, z), delta = 0.08 (nu = 0.04), t = 1, N = 14,000 draws
# per state and iteration (fresh, as the paper resamples), K = 12 iterations,
# tube coefficient, plain estimator; evaluation on 40 x 40 (x, z) slices of
# (-100, 100]^2 at the headings -pi/2, 0 and pi/2.
ROCKET_HEADINGS = (-PI / 2, 0.0, PI / 2)
C7 = Workload("c7_rockets_n3", n=3, ham="rockets", ham_p=(64.0, 32.0, 1.0), datum="ball", datum_p=(2, 1.5),
              nu=0.04, t=1.0, Q=1600, N=14000, K=12, box=((-100.0, 100.0), (-100.0, 100.0), (-PI / 2, PI / 2)),
              tilt=False, sample_mode="fresh", cfg=9, tube=True)


def rocket_slice(theta: float, m: int = 40) -> np.ndarray:
    """States of an m x m (x, z) slice of (-100, 100]^2 at heading theta, float32 [m*m, 3]."""
    g = -100.0 + 200.0 * (np.arange(m) + 1) / m
    X, Z = np.meshgrid(g, g)
    return np.stack([X.ravel(), Z.ravel(), np.full(m * m, theta)], 1).astype(np.float32)


# The paper's double integral plant (appendix; Table double_integrator_
# convergence): x1' = x2, x2' = u, |u| <= 1, the control minimising
# H = p1 x1' + p2 x2' (H = p1 x2 - |p2|); target the disc of radius 0.2 about
# the origin (the paper gives no radius); delta = 0.08 (nu = 0.04), N = 8,000
# fresh draws per state and iteration, K = 15, plain estimator (Algorithm 1);
# evaluation on a 128 x 128 grid of [-1, 1]^2 (the range of the paper's
# trajectory figure); the table's backward times t = 0.8, 0.5, 0.2, 0.0 are
# read as the horizons 1 - t (a horizon of 0 would leave v = l exactly).
DINT_TIMES = (0.8, 0.5, 0.2, 0.0)
C9 = Workload("c9_double_integrator_n2", n=2, ham="double_integrator", ham_p=(1.0, -1.0), datum="ball",
              datum_p=(2, 0.2), nu=0.04, t=1.0, Q=16384, N=8000, K=15, box=((-1.0, 1.0), (-1.0, 1.0)),
              tilt=False, sample_mode="fresh", cfg=11)


def dint_grid(m: int = 128) -> np.ndarray:
    """States of an m x m grid of [-1, 1]^2 (cell centres), float32 [m*m, 2]."""
    g = -1.0 + 2.0 * (np.arange(m) + 0.5) / m
    X, V = np.meshgrid(g, g, indexing="ij")
    return np.stack([X.ravel(), V.ravel()], 1).astype(np.float32)


def horizons(w: Workload):
    """Time-to-go of each horizon: t_j = j T / S_t, j = 1..S_t."""
    return [w.T * (j + 1) / w.time_steps for j in range(w.time_steps)]


# 256 problems of stacked decoupled Dubins pairs (n = 3m, m ~ U{1..16}),
# N log-uniform in [4,096, 262,144] and Q log-uniform in [1,024, 65,536]
# (multiples of 256), nu log-uniform in [1e-3, 1e-1], K ~ U{3..8}, t = 1,
# bfloat16 common draws, tube coefficient, Laplace shift.
@dataclass
class BatchProblem:
    w: Workload
    problem_id: int


def c3_batch(P: int = 256, scale: float = 1.0, trial: int = 0):
    """The uneven batch; `scale` < 1 shrinks N and Q (for tests), keeping the spread."""
    g = rng(3, trial)
    out = []
    for p in range(P):
        m = int(g.integers(1, 17))
        N = int(np.exp(g.uniform(np.log(4096), np.log(262144))) * scale) // 256 * 256
        Q = int(np.exp(g.uniform(np.log(1024), np.log(65536))) * scale) // 256 * 256
        nu = float(np.exp(g.uniform(np.log(1e-3), np.log(1e-1))))
        K = int(g.integers(3, 9))
        w = Workload(f"c3_p{p}", n=3 * m, ham="dubins_pairs", datum="min_pair_disks", datum_p=(0.5,), nu=nu, t=1.0,
                     Q=max(Q, 256), N=max(N, 256), K=K, box=dubins_box(m), tilt=True, sample_mode="crn_step",
                     sample_bf16=True, cfg=3, tube=True)
        out.append(BatchProblem(w, p))
    return out


def c3_fields(bp: BatchProblem) -> dict:
    f = bp.w.problem_fields()
    f["seed"] = philox_seed(3) + 1000 * bp.problem_id
    return f


# Time marching with the surrogate as the datum (semigroup form): the n = 3
# Dubins tube workload marched over its ten horizons, and the exact Cole-Hopf
# case H = |p|^2/2, l = |x|^2/2 (closed form at every time) marched the same
# way.  Labels on 16,384 training states per step (N = 4,096, K = 3); a
# 3 x 128 SiLU network trained 30 epochs per step on all labels so far; the
# last step evaluated at the workload's 65,536 states.
TUBE_MARCH = dict(train_states=16384, N=4096, K=3, width=128, depth=3, epochs=30, batch=1024, lr=2e-3,
                  lr_min=1e-4)
# Reach-avoid variant of the n = 3 Dubins tube: the avoid set is the union of
# two discs of radius 0.6 in the relative plane (the heading is free).
AVOID_DISCS = ((1.5, 0.0), (-1.0, -1.2))
AVOID_RADIUS = 0.6
Q3 = Workload("q3_quadratic_n3", n=3, ham="quadratic", datum="half_sqnorm", nu=0.05, t=1.0, Q=65536, N=65536,
              K=1, box=((-2.0, 2.0),) * 3, tilt=True, sample_mode="crn_step", cfg=8, time_steps=10, T=1.0)


# The paper's murmuration study (appendix, simulation setup): 99,996 starlings
# in six flocks of 16,666, seven pursuers on a ring of radius 1.15 about the
# flock centre, capture radius 0.6 (union of capture cylinders), delta = 0.18
# (nu = 0.09), N = 1,600 draws per state, at most seven Picard passes with
# relative tolerance 1e-5, slices 128 x 128 over [-3.5, 3.5]^2 at altitude 0
# and heading 0 at 18 times of the horizon [0, 2], smoothed with a Gaussian of
# 1.5 cells before the topology is read.  Readings (unstated in the paper):
# speeds v_e = v_p = 1 (its special case), turn rates w_e = w_p = 1, climb
# bounds g_lo = -0.25, g_hi = 0.25, plain estimator, tube coefficient, birds
# uniform over the window with altitude in [-0.5, 0.5] and heading in
# [-pi, pi), one query stream per flock; common draws per horizon (with fresh
# draws per state the sampling error is spatially white and the 1.5-cell
# smoothing leaves speckle components in the later slices).
MURMUR_FLOCKS, MURMUR_BIRDS = 6, 16666
MURMUR_RING, MURMUR_PURSUERS, MURMUR_WINDOW, MURMUR_SMOOTH = 1.15, 7, 3.5, 1.5
C8 = Workload("c8_murmuration_n4", n=4, ham="murmuration", ham_p=(1.0, 1.0, 1.0, 1.0, -0.25, 0.25),
              datum="disc_union", datum_p=(0.6, 7), nu=0.09, t=2.0, Q=MURMUR_FLOCKS * MURMUR_BIRDS, N=1600, K=7,
              box=((-3.5, 3.5), (-3.5, 3.5), (-0.5, 0.5), (-PI, PI)), tilt=False, sample_mode="crn_step", cfg=10,
              time_steps=18, T=2.0, tube=True)


def murmuration_centres() -> np.ndarray:
    """The pursuers' planar positions, float32 [7, 2]."""
    a = 2.0 * PI * np.arange(MURMUR_PURSUERS) / MURMUR_PURSUERS
    return np.stack([MURMUR_RING * np.cos(a), MURMUR_RING * np.sin(a)], 1).astype(np.float32)


def starlings() -> np.ndarray:
    """All birds' relative states, float32 [99,996, 4], flock by flock."""
    return np.concatenate([queries(C8, Q=MURMUR_BIRDS, trial=f) for f in range(MURMUR_FLOCKS)])


def murmuration_window(m: int = 128) -> np.ndarray:
    """States of the m x m slice over [-3.5, 3.5]^2 at altitude 0 and heading 0, float32 [m*m, 4]."""
    g = np.linspace(-MURMUR_WINDOW, MURMUR_WINDOW, m)
    X, Y = np.meshgrid(g, g)
    return np.stack([X.ravel(), Y.ravel(), np.zeros(m * m), np.zeros(m * m)], 1).astype(np.float32)
