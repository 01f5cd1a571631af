"""Philox4x64-10 counter-based generator, plain numpy -- TEST INFRASTRUCTURE
ONLY (tests, smoke and the benchmark's CPU leg).

Definition (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11, the Philox family): a 256-bit counter x = (x0, x1, x2, x3)
and a 128-bit key k = (k0, k1) of 64-bit words go through ten rounds; round
r (r = 0..9) uses the key bumped r times by the Weyl constants
(W0, W1) = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B) and maps
    (hi0, lo0) = M0 * x0,  (hi1, lo1) = M1 * x2     (128-bit products)
    x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)
with M0 = 0xD2E7470EE14C6C93 and M1 = 0xCA5A826395121157.  The four output
words are the counter after the tenth round.

Factors of the request workload draw from it as follows: element e of the
column-major n x n factor number j of client c is word (e mod 4) of
philox((e div 4, j, 0, 0), (seed, c)), mapped to (w >> 11) 2^-53 in [0, 1),
then 2 u - 1 in [-1, 1) (exact), then multiplied by the scale given by the
caller (a binary64 value, one rounding).

Parity status: pinned against numpy's independent Philox4x64-10 bit generator
in tests/test_oracle_philox.py.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK = (1 << 64) - 1


def philox(counter, key, rounds: int = 10):
    """One block: four 64-bit words from a 4-word counter and a 2-word key
    (Python ints)."""
    x0, x1, x2, x3 = (int(v) & MASK for v in counter)
    k0, k1 = (int(v) & MASK for v in key)
    for _ in range(rounds):
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK
        hi1, lo1 = p1 >> 64, p1 & MASK
        x0, x1, x2, x3 = (hi1 ^ x1 ^ k0) & MASK, lo1, (hi0 ^ x3 ^ k1) & MASK, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return x0, x1, x2, x3


def words_to_uniform(w):
    """64-bit words -> binary64 values in [-1, 1): 2 ((w >> 11) 2^-53) - 1."""
    w = np.asarray(w, dtype=np.uint64)
    u = (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return 2.0 * u - 1.0


def factor(seed: int, client: int, j: int, n: int, scale: float) -> np.ndarray:
    """Factor number j of a client: (n, n) ordinary matrix (row r, column c is
    element e = c n + r of the column-major storage)."""
    total = n * n
    words = np.empty(((total + 3) // 4) * 4, dtype=np.uint64)
    for b in range((total + 3) // 4):
        words[4 * b:4 * b + 4] = philox((b, j, 0, 0), (seed, client))
    vals = words_to_uniform(words[:total]) * scale
    return vals.reshape(n, n).T.copy()      # storage is column-major
