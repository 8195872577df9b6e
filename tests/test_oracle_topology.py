"""Pins of the topology oracle on hand-built slices whose topology is plain
(no diagonal contacts): a disc, two discs, a ring, a ring with two holes, a
hole open to the border, the empty and the full grid; a diagonal contact,
which 4-connectivity splits; and the three event rules on a hand-made
sequence."""
import numpy as np

from oracle import topology


def grid(n=64):
    y, x = np.mgrid[0:n, 0:n]
    return x.astype(float), y.astype(float)


def disc(cx, cy, r, n=64):
    x, y = grid(n)
    return np.hypot(x - cx, y - cy) - r


def test_plain_shapes():
    assert topology.markers(disc(32, 32, 10)) == (1, 0, 1)
    two = np.minimum(disc(15, 32, 8), disc(48, 32, 8))
    assert topology.markers(two) == (2, 0, 2)
    ring = np.maximum(disc(32, 32, 20), -disc(32, 32, 8))              # annulus: v <= 0 between radii
    assert topology.markers(ring) == (1, 1, 0)
    two_holes = np.maximum(np.maximum(disc(32, 32, 26), -disc(22, 32, 6)), -disc(42, 32, 6))
    assert topology.markers(two_holes) == (1, 2, -1)
    open_hole = np.maximum(disc(0, 32, 30), -disc(0, 32, 10))          # half annulus cut by the border
    assert topology.markers(open_hole) == (1, 0, 1)
    assert topology.markers(np.ones((16, 16))) == (0, 0, 0)
    assert topology.markers(-np.ones((16, 16))) == (1, 0, 1)


def test_diagonal_contact_is_two_components():
    v = np.ones((6, 6))
    v[1:3, 1:3] = -1
    v[3:5, 3:5] = -1                                                    # corners touch at one point
    assert topology.markers(v)[0] == 2


def test_event_rules():
    chi = [1, 1, 0, 2, 1]
    beta1 = [0, 0, 1, 0, 1]
    ncomp = [1, 1, 1, 2, 2]
    ev = topology.events(chi, beta1, ncomp)
    assert ev.tolist() == [0, 0, topology.VACUOLE | topology.CORDON, topology.FRAGMENTATION,
                           topology.VACUOLE | topology.CORDON]
