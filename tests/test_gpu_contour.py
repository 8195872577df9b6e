"""Marching-squares isocontours on the device against the oracle (runs on an
MI355X): random smooth fields with islands and holes on several grids, a
level other than zero, a circle, the saddle cells, no-cell grids and a
too-small output buffer."""
import numpy as np
import pytest

from oracle import contour as oc
from tests._helpers import to_dev
from tests.test_gpu_topology import smooth_field

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def ordered(seg, sl):
    """Rows sorted by (slice, cell of the midpoint, endpoints) after ordering the endpoints."""
    seg = np.asarray(seg, dtype=np.float64).reshape(-1, 4)
    a, b = seg[:, :2], seg[:, 2:]
    swap = (a[:, 0] > b[:, 0]) | ((a[:, 0] == b[:, 0]) & (a[:, 1] > b[:, 1]))
    lo, hi = np.where(swap[:, None], b, a), np.where(swap[:, None], a, b)
    s = np.concatenate([lo, hi], 1)
    mid = 0.5 * (lo + hi)
    key = np.stack([np.asarray(sl, dtype=np.float64), np.floor(mid[:, 1]), np.floor(mid[:, 0]),
                    np.round(s[:, 0], 3), np.round(s[:, 1], 3)], 1)
    return s[np.lexsort(key.T[::-1])]


def compare(vs, level=0.0):
    from paper_2605_18566_amd import isocontour
    seg, sl = isocontour(to_dev(np.stack(vs)), level)
    got = ordered(seg.cpu().numpy(), sl.cpu().numpy())
    refs = [oc.segments(v, level) for v in vs]
    ref = ordered(np.concatenate(refs), np.concatenate([np.full(len(r), b) for b, r in enumerate(refs)]))
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, atol=2e-4, rtol=0)
    return len(got)


@pytest.mark.parametrize("ny,nx,B,level", [(128, 128, 8, 0.0), (37, 53, 12, 0.0), (64, 96, 6, 0.15)])
def test_random_fields_match_oracle(ny, nx, B, level):
    rng = np.random.default_rng(ny + 7 * nx)
    vs = [smooth_field(rng, ny, nx, holes=b % 2 == 1) for b in range(B)]
    n = compare(vs, level)
    print(f"[{ny}x{nx} level {level}] {n} segments", flush=True)


def test_circle_and_saddles():
    y, x = np.mgrid[0:128, 0:128].astype(np.float32)
    circle = np.hypot(x - 64.2, y - 61.7) - 37.3
    saddles = np.zeros((128, 128), dtype=np.float32) + 1.0
    saddles[10:12, 10:12] = [[-1.0, 0.5], [0.5, -1.0]]                  # centre inside
    saddles[20:22, 20:22] = [[-0.5, 1.0], [1.0, -0.5]]                  # centre outside
    compare([circle.astype(np.float32), saddles])


def test_degenerate_grids_and_small_buffer():
    from paper_2605_18566_amd import _lib, isocontour
    seg, sl = isocontour(to_dev(np.array([[[-1.0]]], dtype=np.float32)))
    assert seg.shape[0] == 0
    y, x = np.mgrid[0:64, 0:64].astype(np.float32)
    v = to_dev(np.hypot(x - 32, y - 32) - 20)
    full, _ = isocontour(v)
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    buf = torch.full((10, 4), -7.0, device="cuda")
    assert _lib.lib().hjg_isocontour(1, 64, 64, v.data_ptr(), 0.0, buf.data_ptr(), None, 10, count.data_ptr(),
                                     None) == 0
    assert int(count.item()) == full.shape[0] > 10
    assert bool((buf != -7.0).all())                        # exactly the first 10 slots written
