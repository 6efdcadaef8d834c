"""Word and min/max operations of the Loefdahl-Scharmer filter kernel,
written out in Python and checked against plain definitions.

The 64x64 island search of the filter works on one
64-bit word per grid row: each sweep ORs in the rows above and below, the
periodic neighbours within the row, and the runs of the row by a doubling
fill, until no word changes.  Here the same word operations, written out in
Python, are checked against a breadth-first search of the 4-connected
component of the zero frequency on the periodic grid, on random masks and
on disk-like masks of the kind the filter produces."""
from collections import deque

import numpy as np

MASK = (1 << 64) - 1
N = 64


def _fill_up(x, m):
    s = 1
    while s < 64:
        x |= m & ((x << s) & MASK)
        m &= (m << s) & MASK
        s <<= 1
    return x


def _fill_down(x, m):
    s = 1
    while s < 64:
        x |= m & (x >> s)
        m &= m >> s
        s <<= 1
    return x


def island_words(B):
    M = [sum(1 << x for x in range(N) if B[y, x]) for y in range(N)]
    L = [0] * N
    L[0] = M[0] & 1
    for _ in range(N * N):
        new = []
        for y in range(N):
            x = L[y] | ((L[(y - 1) % N] | L[(y + 1) % N]) & M[y])
            x |= (((x << 1) & MASK) | (x >> 63) | (x >> 1) | ((x << 63) & MASK)) & M[y]
            new.append(_fill_down(_fill_up(x, M[y]), M[y]))
        changed = new != L
        L = new
        if not changed:
            break
    return np.array([[(L[y] >> x) & 1 for x in range(N)] for y in range(N)], bool)


def island_bfs(B):
    out = np.zeros_like(B, bool)
    if not B[0, 0]:
        return out
    q = deque([(0, 0)])
    out[0, 0] = True
    while q:
        y, x = q.popleft()
        for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            yy, xx = (y + dy) % N, (x + dx) % N
            if B[yy, xx] and not out[yy, xx]:
                out[yy, xx] = True
                q.append((yy, xx))
    return out


def test_row_word_fill_matches_breadth_first_search():
    rng = np.random.default_rng(0)
    f = np.fft.fftfreq(N) * N
    r2 = f[:, None] ** 2 + f[None, :] ** 2
    for t in range(60):
        if t % 2:
            B = rng.random((N, N)) < rng.uniform(0.3, 0.8)
        else:
            B = ((r2 < rng.uniform(50, 900)) & (rng.random((N, N)) < 0.95)) | (
                rng.random((N, N)) < 0.05)
        if t % 7 == 0:
            B[0, 0] = False
        np.testing.assert_array_equal(island_words(B), island_bfs(B), err_msg=str(t))
    # a spiral corridor: many sweeps, runs that wrap around the row ends
    B = np.zeros((N, N), bool)
    B[0, :] = True
    B[:, N - 1] = True
    B[N - 1, 2:] = True
    B[2:, 2] = True
    B[2, 2:N - 3] = True
    B[5, 40] = True   # isolated
    np.testing.assert_array_equal(island_words(B), island_bfs(B))


def _med3(a, b, c):
    return np.maximum(np.minimum(a, b), np.minimum(np.maximum(a, b), c))


def median9_by_triples(v):
    """The kernel's median of nine: sort each triple, then the median of
    (largest low, median middle, smallest high)."""
    lo, mi, hi = [], [], []
    for t in range(3):
        a, b, c = v[3 * t], v[3 * t + 1], v[3 * t + 2]
        lo_ab, hi_ab = np.minimum(a, b), np.maximum(a, b)
        lo.append(np.minimum(lo_ab, c))
        mi.append(np.maximum(lo_ab, np.minimum(hi_ab, c)))
        hi.append(np.maximum(hi_ab, c))
    return _med3(np.maximum(np.maximum(lo[0], lo[1]), lo[2]), _med3(*mi),
                 np.minimum(np.minimum(hi[0], hi[1]), hi[2]))


def test_median_of_nine_by_triples_is_the_median():
    rng = np.random.default_rng(1)
    for trial in range(6):
        if trial % 3 == 0:   # clipped filter values: many exact zeros and ones
            v = rng.random((9, 50000)).astype(np.float32)
            v[v < 0.3] = 0.0
            v[v > 0.9] = 1.0
        else:                # small integers: many ties
            v = rng.integers(0, 4 if trial % 2 else 1000, size=(9, 50000)).astype(np.float32)
        np.testing.assert_array_equal(median9_by_triples(v), np.sort(v, axis=0)[4])
