"""Pins for the Philox4x64-10 oracle (oracle/philox.py) against numpy's
independent implementation of the same generator, and for the mapping of its
words to factor matrices."""
import numpy as np
import pytest

from oracle import philox as P


def _numpy_blocks(key, counter, blocks):
    """numpy's Philox bit generator advances its 256-bit counter before each
    block of four words."""
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(counter, dtype=np.uint64))
    return [int(w) for w in bg.random_raw(4 * blocks)]


@pytest.mark.parametrize("key,counter", [
    ((0, 0), (0, 0, 0, 0)),
    ((1, 2), (5, 0, 0, 0)),
    ((2 ** 64 - 1, 12345), (2 ** 64 - 1, 7, 3, 9)),        # carry into the second word
    ((0xDEADBEEF, 0), (17, 2 ** 63, 0, 1)),
    ((3, 0x9E3779B97F4A7C15), (2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 1, 5)),
])
def test_matches_numpy_philox(key, counter):
    c = sum(v << (64 * i) for i, v in enumerate(counter))
    ours = []
    for b in range(3):
        cc = (c + 1 + b) % (1 << 256)
        ours += P.philox([(cc >> (64 * i)) & P.MASK for i in range(4)], key)
    assert ours == _numpy_blocks(key, counter, 3)


def test_fewer_rounds_differ():
    # every round matters: 9 rounds does not reproduce the 10-round output
    assert P.philox((1, 2, 3, 4), (5, 6), rounds=9) != P.philox((1, 2, 3, 4), (5, 6))


def test_uniform_mapping_exact_and_in_range():
    w = np.array([0, 2 ** 64 - 1, 2 ** 63, 2 ** 11, 2 ** 11 - 1], dtype=np.uint64)
    u = P.words_to_uniform(w)
    assert u[0] == -1.0
    assert u[1] == 1.0 - 2.0 ** -52
    assert u[2] == 0.0
    assert u[3] == -1.0 + 2.0 ** -52
    assert u[4] == -1.0                     # the low 11 bits are dropped


def test_factor_layout_and_moments():
    n, scale = 48, (3.0 / 48) ** 0.5
    F = P.factor(7, 3, 11, n, scale)
    assert F.shape == (n, n)
    # element (r, c) is word e mod 4 of block e div 4, e = c n + r
    for r, c in [(0, 0), (5, 0), (0, 1), (47, 47), (13, 29)]:
        e = c * n + r
        wd = P.philox((e // 4, 11, 0, 0), (7, 3))[e % 4]
        assert F[r, c] == P.words_to_uniform([wd])[0] * scale
    big = P.factor(1, 0, 0, 256, 1.0)
    assert abs(big.mean()) < 0.01
    assert abs(big.var() - 1.0 / 3.0) < 0.01
    # different clients and steps give different factors
    assert not np.array_equal(P.factor(7, 4, 11, n, scale), F)
    assert not np.array_equal(P.factor(7, 3, 12, n, scale), F)
