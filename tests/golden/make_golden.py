"""Writes oracle_reference.txt: reference values computed by the FP64 oracle
alone (no device code), kept so that any later change to the oracle's
arithmetic shows up as a changed number.

    python tests/golden/make_golden.py

Contents (each block cites what it follows):
  * Algorithm 1, one iteration, H = |p|^2/2 (coefficient exactly 1/delta, the
    remark on the exact reduction), disc datum |x| - 1, n = 2, nu = 0.05,
    t = 0.5, with the Laplace shift theta = -sigma^2 c D l(x) (Section 2.4):
    value and Monte-Carlo gradient (log-sum-exp, Monte-Carlo gradient and
    tilted-proposal corollaries) on deterministic equal-weight quantile
    draws (400 x 400 tensor grid), at six states;
  * the same states with the datum |x|^2/2, where the method is exact (the
    closed form |x|^2/(2(1 + t)) + n nu log(1 + t) listed beside it);
  * Philox4x32-10 words (Salmon et al., SC'11) for a few counters and keys.
"""
import os
import sys

import numpy as np
from scipy import special

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import estimator, model, philox  # noqa: E402

STATES = np.array([[0.3, -0.4], [1.0, 0.5], [1.2, 0.3], [-0.7, 0.9], [0.05, 0.02], [1.5, -1.1]])
NU, T, N1 = 0.05, 0.5, 400
COUNTERS = [(0, 0, 0, 0, 0, 0), (1, 2, 3, 4, 5, 6), (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF,
                                                     0xFFFFFFFF), (12345, 0, 7, 0x00050300, 0x66080000, 0x00000260)]


def quantile_draws(n, n1):
    q = special.ndtri((np.arange(n1) + 0.5) / n1)
    mesh = np.meshgrid(*([q] * n), indexing="ij")
    return np.stack([m.ravel() for m in mesh])


def compute():
    z = quantile_draws(2, N1)
    rows = []
    for datum, dp in (("ball", (2, 1.0)), ("half_sqnorm", ())):
        pb = model.Problem(n=2, ham="quadratic", datum=datum, datum_p=dp, nu=NU, tilt=True)
        c = np.full(len(STATES), 1 / pb.delta)
        theta = model.tilt(pb, np.sqrt(pb.delta * T), c, model.datum_grad(pb, STATES))
        est = estimator.value_grad(pb, STATES, T, z.shape[1], c, theta, z=z)
        for q in range(len(STATES)):
            rows.append((datum, q, float(est.v[q]), float(est.grad[q, 0]), float(est.grad[q, 1])))
    words = []
    for c in COUNTERS:
        w = philox.philox4x32_10(np.uint32(c[0]), np.uint32(c[1]), np.uint32(c[2]), np.uint32(c[3]), c[4], c[5])
        words.append(tuple(int(np.asarray(x).ravel()[0]) for x in w))
    return rows, words


def main():
    rows, words = compute()
    path = os.path.join(HERE, "oracle_reference.txt")
    with open(path, "w") as f:
        f.write("# Written by tests/golden/make_golden.py from oracle/ only.\n")
        f.write(f"# estimator: n = 2, H = |p|^2/2, nu = {NU}, t = {T}, quantile draws {N1} x {N1}\n")
        f.write("# estimate datum state v dv/dx0 dv/dx1\n")
        for datum, q, v, g0, g1 in rows:
            f.write(f"estimate {datum} {q} {v!r} {g0!r} {g1!r}\n")
        f.write("# philox c0 c1 c2 c3 k0 k1 -> w0 w1 w2 w3\n")
        for c, w in zip(COUNTERS, words):
            f.write("philox " + " ".join(str(x) for x in c) + " -> " + " ".join(str(x) for x in w) + "\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
