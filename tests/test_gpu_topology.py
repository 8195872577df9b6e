"""Topology markers on the device against the oracle (scipy labelling), on an
MI355X: hand-built shapes, batches of random smooth fields at several grid
sizes (ragged, 1 x 1, the 128 x 128 maximum), diagonal contacts, and the
size limit."""
import numpy as np
import pytest

from oracle import topology as ot
from tests._helpers import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def smooth_field(rng, ny, nx, blobs=12, holes=False):
    # islands in an outside sea, or (holes) an inside sea with raised bumps
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    base, sign = (-0.4, -1.0) if holes else (0.6, 1.0)
    v = np.full((ny, nx), base)
    for _ in range(blobs + 8 * holes):
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        s = rng.uniform(1.5, 0.2 * max(nx, ny) + 2)
        v -= sign * rng.uniform(-0.8, 1.2) * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * s * s))
    return v.astype(np.float32)


def run(vs):
    from paper_2605_18566_amd import topology
    nc, b1, chi = topology(to_dev(np.stack(vs)))
    return nc.cpu().numpy(), b1.cpu().numpy(), chi.cpu().numpy()


@pytest.mark.parametrize("ny,nx,B", [(128, 128, 24), (37, 53, 40), (1, 1, 3), (1, 100, 5), (128, 1, 5), (64, 96, 16)])
def test_random_fields_match_oracle(ny, nx, B):
    rng = np.random.default_rng(ny * 1000 + nx)
    vs = [smooth_field(rng, ny, nx, holes=b % 2 == 1) for b in range(B)]
    if ny * nx == 1:
        vs = [np.array([[v]], dtype=np.float32) for v in (-1.0, 0.0, 1.0)]
    nc, b1, chi = run(vs)
    ref = np.array([ot.markers(v) for v in vs])
    np.testing.assert_array_equal(nc, ref[:, 0])
    np.testing.assert_array_equal(b1, ref[:, 1])
    np.testing.assert_array_equal(chi, ref[:, 2])
    print(f"[{ny}x{nx}] n_comp {nc.min()}..{nc.max()}, beta1 {b1.min()}..{b1.max()}", flush=True)


def test_hand_built_shapes_and_diagonals():
    y, x = np.mgrid[0:128, 0:128].astype(float)
    d = lambda cx, cy, r: np.hypot(x - cx, y - cy) - r
    shapes = [d(64, 64, 20), np.maximum(d(64, 64, 50), -d(64, 64, 20)),
              np.maximum(np.maximum(d(64, 64, 55), -d(44, 64, 12)), -d(84, 64, 12)),
              np.maximum(d(0, 64, 60), -d(0, 64, 20)), np.ones((128, 128)), -np.ones((128, 128))]
    checker = np.where((x.astype(int) + y.astype(int)) % 2 == 0, -1.0, 1.0)   # every inside cell alone
    shapes.append(checker)
    vs = [s.astype(np.float32) for s in shapes]
    nc, b1, chi = run(vs)
    ref = np.array([ot.markers(v) for v in vs])
    np.testing.assert_array_equal(np.stack([nc, b1, chi], 1), ref)
    assert nc[-1] == 128 * 128 // 2


def test_size_limit_and_nan():
    from paper_2605_18566_amd import _lib, topology
    with pytest.raises(_lib.HJGError):
        topology(torch.zeros((1, 129, 128), device="cuda"))
    v = np.ones((20, 20), dtype=np.float32)
    v[5:10, 5:10] = np.nan                                  # NaN counts as outside
    v[12:15, 12:15] = -1
    nc, b1, _ = run([v])
    assert (nc[0], b1[0]) == ot.markers(np.nan_to_num(v, nan=1.0))[:2]
