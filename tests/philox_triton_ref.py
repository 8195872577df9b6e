"""Philox4x32-10 words from Triton's own implementation, run on the CPU.

An independent implementation of the cipher for pinning the oracle's
generator: Triton's ``tl.random.philox`` (its language library, executed by
the CPU interpreter, ``TRITON_INTERPRET=1``).  Run as a child process by
tests/test_oracle_philox.py, because the interpreter switch must be set before
Triton is imported.  Reads a JSON list of cases on stdin, each
``{"seed": s, "c0": [..], "c1": x, "c2": y, "c3": z}`` (c0 a list of counter
words, the others scalars), and prints the four output words of every counter
as a JSON list of lists.  Nothing in the library imports this file.
"""
import json
import os
import sys

os.environ["TRITON_INTERPRET"] = "1"

import torch  # noqa: E402
import triton  # noqa: E402
import triton.language as tl  # noqa: E402


@triton.jit
def _words(out, cp, seed, G: tl.constexpr):
    i = tl.arange(0, G)
    c0 = tl.load(cp + 4 * i)
    c1 = tl.load(cp + 4 * i + 1)
    c2 = tl.load(cp + 4 * i + 2)
    c3 = tl.load(cp + 4 * i + 3)
    a, b, c, d = tl.random.philox(seed, c0, c1, c2, c3, 10)
    tl.store(out + 4 * i, a)
    tl.store(out + 4 * i + 1, b)
    tl.store(out + 4 * i + 2, c)
    tl.store(out + 4 * i + 3, d)


def main():
    cases = json.load(sys.stdin)
    res = []
    for cs in cases:
        c0 = [int(v) & 0xFFFFFFFF for v in cs["c0"]]
        G = 1
        while G < len(c0):
            G *= 2
        c0 = c0 + [0] * (G - len(c0))
        ctr = []
        for v in c0:
            ctr += [v, int(cs["c1"]) & 0xFFFFFFFF, int(cs["c2"]) & 0xFFFFFFFF, int(cs["c3"]) & 0xFFFFFFFF]
        # counter words as uint32 tensors (a Python integer above 2^31 would
        # enter the kernel as a 64-bit scalar); tl.random.philox splits the
        # 64-bit seed into its (low, high) key words
        ctrt = torch.tensor(ctr, dtype=torch.int64).to(torch.uint32)
        out = torch.zeros(4 * G, dtype=torch.uint32)
        _words[(1,)](out, ctrt, int(cs["seed"]) & 0xFFFFFFFFFFFFFFFF, G)
        w = out.to(torch.int64).tolist()
        res.append([w[4 * g:4 * g + 4] for g in range(len(cs["c0"]))])
    json.dump(res, sys.stdout)


if __name__ == "__main__":
    main()
