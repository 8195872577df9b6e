"""The oracle against its stored reference values (tests/golden/
oracle_reference.txt, written by tests/golden/make_golden.py from oracle/
only): a changed number means the oracle's arithmetic changed.  The exact
quadratic rows are also held to the closed form of the viscous equation, so
the file itself is pinned."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402


def read_reference():
    est, phx = {}, []
    for line in open(os.path.join(HERE, "golden", "oracle_reference.txt")):
        if line.startswith("estimate "):
            _, datum, q, v, g0, g1 = line.split()
            est[(datum, int(q))] = (float(v), float(g0), float(g1))
        elif line.startswith("philox "):
            lhs, rhs = line[len("philox "):].split("->")
            phx.append((tuple(int(x) for x in lhs.split()), tuple(int(x) for x in rhs.split())))
    return est, phx


def test_oracle_reproduces_its_reference_values():
    est, phx = read_reference()
    rows, words = make_golden.compute()
    assert len(rows) == len(est) == 12 and len(words) == len(phx) == 4
    for datum, q, v, g0, g1 in rows:
        np.testing.assert_allclose((v, g0, g1), est[(datum, q)], rtol=1e-10, atol=1e-13)
    for (c, w_ref), w in zip(phx, words):
        assert tuple(c) == tuple(make_golden.COUNTERS[phx.index((c, w_ref))]) and tuple(w) == w_ref


def test_reference_file_meets_the_closed_form():
    est, _ = read_reference()
    x, t, nu = make_golden.STATES, make_golden.T, make_golden.NU
    v_cf = np.sum(x * x, 1) / (2 * (1 + t)) + 2 * nu * np.log1p(t)
    for q in range(len(x)):
        v, g0, g1 = est[("half_sqnorm", q)]
        # quadrature of the tilted estimator: 4e-5 in v, 7.5e-4 in the gradient
        assert abs(v - v_cf[q]) <= 1e-4
        np.testing.assert_allclose((g0, g1), x[q] / (1 + t), atol=1e-3)
