"""FP64 CPU oracle for the HJ-Gauss Monte-Carlo Picard sweep.

TEST INFRASTRUCTURE.  Plain, slow, obviously correct numpy code written from
the paper (Algorithm 1; the log-sum-exp, Monte-Carlo gradient and
tilted-proposal corollaries; the coefficient definition, its regularisation and
clipping).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
device path; the Gaussian draws come from its own Philox4x32-10
implementation (``oracle.philox``).

Parity status per function (what pins it, see tests/test_oracle_*.py):
  philox.philox4x32_10 / normals : word for word against an independent
                                   implementation (Triton's philox, run by its
                                   CPU interpreter) over several keys and all
                                   four counter words; structural and
                                   statistical tests
  estimator.value_grad           : closed forms (quadratic H with quadratic and
                                   linear data), 1D folded-normal closed form,
                                   2D disk quadrature, finite-difference grid
                                   solves of the PDE in 1D and 2D, c -> 0 limit, tilt
                                   invariance, Stein vs finite differences,
                                   N^-1/2 rate
  estimator.picard               : quadratic-H fixed point in one step,
                                   deterministic contraction under common
                                   random numbers; the warm start v0 (zero
                                   first residual at a p-independent fixed
                                   point, NaN starts flagged); for non-quadratic H the
                                   Picard fixed point is "parity unpinned"
                                   against the viscous solution (the paper's
                                   quasi-linearisation defect is not computable)
  estimator.tube_step            : semigroup step reproduces the closed form of
                                   the exact quadratic case at the later time;
                                   from t_prev = 0 with the terminal datum it
                                   is bit-identical to estimator.picard
  mlp.forward_bf16_storage /     : reduces to the plain forward when rounding
    value_at, round_bf16           is the identity; rounding ties by hand and
                                   against the draw generator's rounding
  certify.classify / mc_margin / : the corollary's sign guarantee as a property;
    error_budget                   the margin inverts the tail bound, has
                                   Hoeffding's c -> 0 limit and covers the
                                   exact quadratic case over 200 draw sets
  topology.markers / events      : hand-built slices of plain topology (discs,
                                   rings, holes open to the border, diagonal
                                   contact) and a hand-made event sequence
  avoid.project                  : the reach-avoid property (no avoid-set state
                                   reached), lattice property of the maximum,
                                   brute-force obstacle level, projected
                                   gradient vs central differences, idempotence
  contour.segments               : exact on linear fields, circle length and
                                   radius, the two saddle cells by hand
  model.hamiltonian (Dubins,     : brute-force max-min over control grids
    multi-pursuer game)
  model.coefficient /            : the general branch gives exactly 1/delta for
    frozen_coefficient             H = |p|^2/2 with eta = 0; hand-worked Dubins
                                   values (both signs of the p2 term, tube
                                   form); sign-keeping clip
  model.datum (capture)          : a hand-built configuration; its gradient
                                   against central differences
  model.datum / datum_grad       : a brute-force loop over pairs (m = 1..15,
    (min_pair_disks)               r = 0), central differences, ties to the
                                   lowest pair and the centre kink by hand
  knn.knn                        : a k-d tree (scipy) on random points, the
                                   unit-lattice closed form, duplicate points
                                   and float32 near-ties
"""
