"""Pins of the oracle's Philox4x32-10 draws (CPU only).

The generator is pinned by (i) word-for-word agreement with an independent
implementation of Philox4x32-10, Triton's ``tl.random.philox`` run by its CPU
interpreter (tests/philox_triton_ref.py), over several keys and all four
counter words; (ii) structural properties any correct counter-based bijection
has; (iii) the exact uniform and Box-Muller mapping at extreme words; (iv)
statistical tests of the normals; and (v) bit agreement with the device
implementation (GPU tests).
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import philox


def test_uniform_mapping_extremes():
    w = np.array([0, 0xFF, 0x100, 0xFFFFFFFF], dtype=np.uint64)
    ua = philox.uniform_open_closed(w)
    ub = philox.uniform_closed_open(w)
    assert ua.tolist() == [2.0 ** -24, 2.0 ** -24, 2.0 * 2.0 ** -24, 1.0]
    assert ub.tolist() == [0.0, 0.0, 2.0 ** -24, 1.0 - 2.0 ** -24]
    # all uniforms are exactly representable in FP32
    assert np.all(ua.astype(np.float32).astype(np.float64) == ua)


def test_box_muller_at_known_angles():
    # angle word giving u_b = 1/4 -> phi = pi/2: (0, r); radius word giving u_a = 1 -> r = 0
    wb = np.uint64((1 << 22) << 8)
    z0, z1 = philox.box_muller(np.uint64(0xFFFFFFFF), wb)
    assert abs(z0) == 0.0 and z1 == 0.0
    wa = np.uint64(0)                       # u_a = 2^-24 -> r = sqrt(48 ln 2)
    z0, z1 = philox.box_muller(wa, np.uint64(0))
    assert np.isclose(z0, np.sqrt(48 * np.log(2.0)), rtol=1e-15) and z1 == 0.0


def test_round_is_a_permutation_on_distinct_counters():
    # a Philox round is a bijection of the 128-bit block for a fixed key:
    # distinct counters never collide.
    g = np.arange(1 << 16, dtype=np.uint64)
    w = philox.philox4x32_10(g, 0, 7, 3, 0x1234, 0x5678)
    packed = set(zip(*(x.tolist() for x in w)))
    assert len(packed) == 1 << 16


def test_avalanche_single_bit_flip():
    # flipping one counter bit changes about half of the 128 output bits
    rng = np.random.default_rng(0)
    base = rng.integers(0, 2 ** 32, size=(4, 4096), dtype=np.uint64)
    out0 = philox.philox4x32_10(*base, 11, 22)
    flips = []
    for word in range(4):
        for bit in (0, 13, 31):
            b = base.copy()
            b[word] ^= np.uint64(1 << bit)
            out1 = philox.philox4x32_10(*b, 11, 22)
            diff = sum(np.unpackbits((o0 ^ o1).view(np.uint8)).sum() for o0, o1 in zip(out0, out1))
            flips.append(diff / (128 * 4096))
    assert np.all(np.abs(np.array(flips) - 0.5) < 0.01)


def test_key_matters():
    a = philox.philox4x32_10(np.arange(64), 0, 0, 0, 1, 2)
    b = philox.philox4x32_10(np.arange(64), 0, 0, 0, 1, 3)
    assert not np.array_equal(a[0], b[0])


def test_words_uniform_chi2():
    w = philox.philox4x32_10(np.arange(1 << 18), 5, 6, 7, 99, 100)
    for x in w:
        counts = np.bincount((x >> np.uint32(24)).astype(np.int64), minlength=256)
        chi2 = np.sum((counts - counts.mean()) ** 2 / counts.mean())
        assert stats.chi2.sf(chi2, 255) > 1e-4


def test_normals_moments_and_ks():
    z = philox.normals(seed=0x2605185660000, stream=philox.CRN_STREAM, tag=philox.make_tag(3, 1, 0), n=4, N=1 << 16)
    assert z.shape == (4, 1 << 16)
    flat = z.ravel()
    assert abs(flat.mean()) < 5 / np.sqrt(flat.size)
    assert abs(flat.var() - 1) < 5 * np.sqrt(2 / flat.size)
    assert stats.kstest(flat, "norm").pvalue > 1e-4
    c = np.corrcoef(z)
    assert np.all(np.abs(c - np.eye(4)) < 5 / np.sqrt(z.shape[1]))
    # the two members of a Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(z[0, 0::4], z[0, 1::4])[0, 1]) < 5 / np.sqrt(z.shape[1] / 4)


def test_streams_and_tags_independent():
    a = philox.normals(1, 0, philox.make_tag(0, 0, 0), 2, 4096)
    b = philox.normals(1, 1, philox.make_tag(0, 0, 0), 2, 4096)
    c = philox.normals(1, 0, philox.make_tag(0, 0, 1), 2, 4096)
    for u in (b, c):
        r = np.corrcoef(a.ravel(), u.ravel())[0, 1]
        assert abs(r) < 5 / np.sqrt(a.size)


def test_prefix_consistency_and_batched_streams():
    tag = philox.make_tag(2, 3, 4)
    big = philox.normals(7, 5, tag, 3, 103)
    small = philox.normals(7, 5, tag, 3, 50)
    np.testing.assert_array_equal(big[:, :50], small)
    many = philox.normals(7, np.array([4, 5, 6]), tag, 3, 103)
    np.testing.assert_array_equal(many[1], big)


def test_round_bf16_matches_torch_rne():
    # values exactly representable in FP32, so torch's FP32->BF16 rounding
    # (round to nearest, ties to even) is a single rounding, like ours.
    rng = np.random.default_rng(1)
    x = rng.standard_normal(200000).astype(np.float32)
    # include exact ties: FP32 values whose low 16 bits are 0x8000
    ties = (rng.integers(0x3F000000, 0x40800000, 2000).astype(np.uint32) & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    x = np.concatenate([x, ties.view(np.float32), -ties.view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(philox.round_bf16(x.astype(np.float64)), ref)


def test_tag_range_checked():
    with pytest.raises(ValueError):
        philox.make_tag(1 << 16, 0, 0)
    with pytest.raises(ValueError):
        philox.make_tag(0, 256, 0)


# ------------------------------------------------- independent implementation
TRITON_REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "philox_triton_ref.py")


def _triton_words(cases):
    try:
        import triton  # noqa: F401
    except ImportError:
        pytest.skip("Triton (the independent Philox implementation) is not importable")
    r = subprocess.run([sys.executable, TRITON_REF], input=json.dumps(cases), capture_output=True, text=True,
                       timeout=600, cwd=os.path.dirname(TRITON_REF))
    assert r.returncode == 0, r.stderr[-2000:]
    return [np.array(w, dtype=np.uint64).reshape(-1, 4) for w in json.loads(r.stdout)]


def test_words_match_triton_philox():
    """Philox4x32-10 of the oracle equals Triton's implementation word for word.

    The cases cover the 64-bit key split (seed low word = key word 0), keys
    with every bit set, counters whose upper words are all non-zero, the
    common-table stream (0xFFFFFFFF) with real tags, the per-query streams,
    first counter words near 2^32, and the counters of the stored reference
    words.
    """
    rng = np.random.default_rng(2605)
    seeds = [0, 1, 0x0002605185660010, 0xFFFFFFFFFFFFFFFF, 0x8000000000000001, int(rng.integers(0, 2 ** 63))]
    cases = []
    for s in seeds:
        cases.append({"seed": s, "c0": list(range(16)), "c1": 0, "c2": 0xFFFFFFFF, "c3": philox.make_tag(2, 1, 0)})
        cases.append({"seed": s, "c0": [int(v) for v in rng.integers(0, 2 ** 32, 16)],
                      "c1": int(rng.integers(0, 2 ** 32)), "c2": int(rng.integers(0, 2 ** 32)),
                      "c3": int(rng.integers(0, 2 ** 32))})
        cases.append({"seed": s, "c0": [0xFFFFFFFF - i for i in range(8)], "c1": 44, "c2": 65535,
                      "c3": philox.make_tag(255, 9, 254)})
    for c in ((0, 0, 0, 0, 0, 0), (1, 2, 3, 4, 5, 6), (12345, 0, 7, 0x00050300, 0x66080000, 0x00000260)):
        cases.append({"seed": c[4] | (c[5] << 32), "c0": [c[0]], "c1": c[1], "c2": c[2], "c3": c[3]})
    ref = _triton_words(cases)
    for cs, w_ref in zip(cases, ref):
        s = int(cs["seed"])
        w = philox.philox4x32_10(np.array(cs["c0"], dtype=np.uint64), cs["c1"], cs["c2"], cs["c3"],
                                 s & 0xFFFFFFFF, s >> 32)
        np.testing.assert_array_equal(np.stack(w, axis=1).astype(np.uint64), w_ref, err_msg=str(cs))


def test_normals_use_the_pinned_words():
    """The draws of one table column are Box-Muller of the pinned words at the
    stream layout's counters (i div 4, d, stream, tag)."""
    seed, tag, d = 0x0002605185660011, philox.make_tag(4, 2, 0), 3
    z = philox.normals(seed, philox.CRN_STREAM, tag, n=5, N=32)
    w = _triton_words([{"seed": seed, "c0": list(range(8)), "c1": d, "c2": philox.CRN_STREAM, "c3": tag}])[0]
    ua = lambda x: ((x >> np.uint64(8)) + np.uint64(1)).astype(np.float64) * 2.0 ** -24   # noqa: E731
    ub = lambda x: (x >> np.uint64(8)).astype(np.float64) * 2.0 ** -24                    # noqa: E731
    r0, p0 = np.sqrt(-2 * np.log(ua(w[:, 0]))), 2 * np.pi * ub(w[:, 1])
    r1, p1 = np.sqrt(-2 * np.log(ua(w[:, 2]))), 2 * np.pi * ub(w[:, 3])
    want = np.stack([r0 * np.cos(p0), r0 * np.sin(p0), r1 * np.cos(p1), r1 * np.sin(p1)], axis=1).ravel()
    np.testing.assert_allclose(z[d], want, rtol=0, atol=1e-15)
