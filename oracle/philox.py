"""Counter-based Gaussian draws for the CPU oracle (FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.

The method draws iid standard normals z_i ~ N(0, I_n) for every evaluation
state and Picard iteration (paper, Remark "Evaluation states vs. Monte Carlo
samples", and the log-sum-exp corollary in the appendix).  The paper does not
say how the draws are produced.  Both sides of the parity check therefore
implement one published counter-based generator, Philox4x32-10 (Salmon,
Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11),
independently, from its definition:

* state: a 128-bit counter (four 32-bit words) and a 64-bit key (two words);
* one round: multiply word 0 by 0xD2511F53 and word 2 by 0xCD9E8D57 as full
  32x32->64 products; the new words are
  (hi(word2 product) ^ word1 ^ key0, lo(word2 product),
   hi(word0 product) ^ word3 ^ key1, lo(word0 product));
* between rounds the key is advanced by the Weyl constants
  (0x9E3779B9, 0xBB67AE85); ten rounds in all.

Stream layout (a definition of this project, shared with the device side by
specification, not by code):

* key = (seed mod 2^32, seed div 2^32)
* the normal for sample i, dimension d uses counter
  (i div 4, d, stream, tag) and takes output normal number (i mod 4);
  stream = query index in FRESH mode and 0xFFFFFFFF in the common-random-number
  modes; tag = (problem_id << 16) | (time_step << 8) | iteration.
* four words (w0, w1, w2, w3) give two Box-Muller pairs:
  u_a = ((w >> 8) + 1) * 2^-24 in (0, 1] from w0 (resp. w2),
  u_b = (w >> 8) * 2^-24 in [0, 1) from w1 (resp. w3),
  r = sqrt(-2 ln u_a), phi = 2 pi u_b, normals (r cos phi, r sin phi).
  The uniforms are exact in FP32 and FP64 and ln 0 never occurs.

Because the counter does not depend on N, sample i is the same for every N
(tables are prefix-consistent).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
CRN_STREAM = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox rounds on arrays of counter words; returns four uint32 arrays."""
    x0 = np.asarray(c0, dtype=np.uint64) & MASK32
    x1 = np.asarray(c1, dtype=np.uint64) & MASK32
    x2 = np.asarray(c2, dtype=np.uint64) & MASK32
    x3 = np.asarray(c3, dtype=np.uint64) & MASK32
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    key0, key1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * x0            # < 2^64: exact in uint64
        p1 = M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x0 = hi1 ^ x1 ^ np.uint64(key0)
        x1 = lo1
        x2 = hi0 ^ x3 ^ np.uint64(key1)
        x3 = lo0
        key0 = (key0 + W0) & 0xFFFFFFFF
        key1 = (key1 + W1) & 0xFFFFFFFF
    return (x0.astype(np.uint32), x1.astype(np.uint32),
            x2.astype(np.uint32), x3.astype(np.uint32))


def make_tag(problem_id: int, time_step: int, iteration: int) -> int:
    if not (0 <= problem_id < 1 << 16 and 0 <= time_step < 1 << 8 and 0 <= iteration < 1 << 8):
        raise ValueError("problem_id < 65536, time_step < 256, iteration < 256 required")
    return (problem_id << 16) | (time_step << 8) | iteration


def split_seed(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def uniform_open_closed(w):
    """((w >> 8) + 1) * 2^-24, a value in (0, 1]."""
    return ((np.asarray(w, dtype=np.uint64) >> np.uint64(8)) + np.uint64(1)).astype(np.float64) * 2.0 ** -24


def uniform_closed_open(w):
    """(w >> 8) * 2^-24, a value in [0, 1)."""
    return (np.asarray(w, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def box_muller(wa, wb):
    """Two FP64 normals from two words (radius word, angle word)."""
    r = np.sqrt(-2.0 * np.log(uniform_open_closed(wa)))
    phi = 2.0 * np.pi * uniform_closed_open(wb)
    return r * np.cos(phi), r * np.sin(phi)


def normals(seed: int, stream, tag: int, n: int, N: int) -> np.ndarray:
    """Standard normals z[d, i] for d < n, i < N (FP64), one stream.

    ``stream`` may be an integer or an array of shape [Q]; the result then has
    shape [Q, n, N].
    """
    k0, k1 = split_seed(seed)
    G = (N + 3) // 4
    g = np.arange(G, dtype=np.uint64)
    d = np.arange(n, dtype=np.uint64)
    s = np.asarray(stream, dtype=np.uint64)
    scalar = s.ndim == 0
    s = s.reshape(-1, 1, 1)
    w0, w1, w2, w3 = philox4x32_10(g[None, None, :], d[None, :, None], s, np.uint64(tag), k0, k1)
    z0, z1 = box_muller(w0, w1)
    z2, z3 = box_muller(w2, w3)
    z = np.stack([z0, z1, z2, z3], axis=-1).reshape(s.shape[0], n, 4 * G)[:, :, :N]
    return z[0] if scalar else z


def round_bf16(x) -> np.ndarray:
    """Round FP64 values to the nearest bfloat16 (8 significant bits), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                 # x = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)


def crn_table(seed: int, problem_id: int, time_step: int, n: int, N: int, bf16: bool = False) -> np.ndarray:
    """The common-random-number table z[d, i] of one (problem, time step)."""
    z = normals(seed, CRN_STREAM, make_tag(problem_id, time_step, 0), n, N)
    return round_bf16(z) if bf16 else z


def fresh_draws(seed: int, problem_id: int, time_step: int, iteration: int, queries, n: int, N: int,
                bf16: bool = False) -> np.ndarray:
    """Fresh draws z[q, d, i] for the given query indices at one Picard iteration."""
    z = normals(seed, np.asarray(queries), make_tag(problem_id, time_step, iteration), n, N)
    return round_bf16(z) if bf16 else z
