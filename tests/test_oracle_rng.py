"""Pins of the reference counter-based generator: the published known-answer
vectors of Philox4x32-10, and the distribution of its Box-Muller normals."""

import os

import numpy as np
from scipy import stats

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "philox4x32_10_kat.txt")


def test_philox_known_answers():
    n = 0
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        assert rng.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])
        n += 1
    assert n == 3


def test_counter_layout():
    # draw i uses word i % 4 of block counter0 + i // 4; the stream id is the
    # upper counter half, the seed the key
    seed, sid = 0x0123456789ABCDEF, 0x0000000100000002
    w = rng.words(seed, sid, 7, 12)
    for t in range(3):
        b = 7 + t
        ref = rng.philox4x32_10((b, 0, 2, 1), (0x89ABCDEF, 0x01234567))
        assert tuple(int(x) for x in w[4 * t:4 * t + 4]) == ref
    # consecutive calls continue one another
    a = rng.words(seed, sid, 7, 8)
    b = rng.words(seed, sid, 9, 4)
    assert np.array_equal(np.concatenate([a, b]), w)


def test_normals_are_standard_normal():
    z = rng.normals(2024, 3, 0, 20000)
    assert abs(z.mean()) < 4.0 / np.sqrt(z.size)
    assert abs(z.std() - 1.0) < 4.0 * np.sqrt(0.5 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # pairs are independent: correlation of cos/sin partners near zero
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 4.0 / np.sqrt(z.size / 2)
