"""Pins of the post-processing oracle (Fourier filters, mosaic) against
closed forms, special cases and independent library routines."""

import numpy as np
import pytest
from scipy import ndimage
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle
from oracle import postprocess as pp


def test_tophat_closed_form():
    N, fd = 64, 20.0
    H = pp.tophat_filter(N, 0.5, 0.7, fd)
    r = pp.frequency_radius(N)
    assert H[0, 0] == 1.0
    assert np.all(H[r <= 10.0] == 1.0) and np.all(H[r >= 14.0] == 0.0)
    # radius 12 bins is the middle of the transition: cos(pi/2) -> 1/2
    assert abs(H[12, 0] - 0.5) < 1e-15 and abs(H[0, N - 12] - 0.5) < 1e-15
    # symmetric under u -> -u and non-increasing in |u|
    np.testing.assert_array_equal(H, np.roll(H[::-1, ::-1], 1, (0, 1)))
    order = np.argsort(r.ravel(), kind="stable")
    assert np.all(np.diff(H.ravel()[order]) <= 1e-15)


def test_identity_filter_gives_the_object():
    rng = np.random.default_rng(1)
    o = rng.standard_normal((16, 16))
    O = oracle.dft2(o)
    H = pp.tophat_filter(16, 100.0, 101.0, 1.0)
    np.testing.assert_allclose(pp.filtered_object(O, H), o, atol=1e-13)


def test_median_matches_scipy():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((24, 24))
    np.testing.assert_array_equal(pp.median3_periodic(x), ndimage.median_filter(x, 3, mode="wrap"))


def _torus_component(mask):
    n0, n1 = mask.shape
    idx = np.arange(n0 * n1).reshape(n0, n1)
    rows, cols = [], []
    for dy, dx in ((1, 0), (0, 1)):
        nb = np.roll(np.roll(idx, -dy, 0), -dx, 1)
        both = mask & np.roll(np.roll(mask, -dy, 0), -dx, 1)
        rows.append(idx[both])
        cols.append(nb[both])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    g = coo_matrix((np.ones(len(r)), (r, c)), shape=(n0 * n1, n0 * n1))
    _, lab = connected_components(g, directed=False)
    return mask & (lab.reshape(n0, n1) == lab[0]) if mask[0, 0] else np.zeros_like(mask)


@pytest.mark.parametrize("density", [0.45, 0.6])
def test_connectivity_matches_graph_components(density):
    rng = np.random.default_rng(int(density * 100))
    for _ in range(5):
        m = rng.random((20, 20)) < density
        m[0, 0] = True
        np.testing.assert_array_equal(pp.connected_to_origin(m), _torus_component(m))
    # an island that touches the origin only across the periodic border
    m = np.zeros((8, 8), bool)
    m[0, 0] = m[7, 0] = m[6, 0] = m[0, 7] = True
    m[3, 3] = True
    k = pp.connected_to_origin(m)
    assert k[6, 0] and k[0, 7] and not k[3, 3]


def test_scharmer_raw_closed_forms():
    """Noise-free frames D_j = O S_j: sum D conj(S) = O sum |S|^2, so the
    unclipped filter is 1 - eta / (|O|^2 sum_j |S_j|^2)."""
    rng = np.random.default_rng(3)
    N, J = 16, 3
    S = rng.standard_normal((1, J, N, N)) + 1j * rng.standard_normal((1, J, N, N))
    O = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    D = O[None, None] * S
    w = np.ones((1, J))
    eta = 0.37
    H = pp.scharmer_raw(D, S, w, [0], eta)
    ref = 1.0 - eta / (np.abs(O) ** 2 * np.sum(np.abs(S[0]) ** 2, axis=0))
    np.testing.assert_allclose(H, ref, rtol=1e-12)
    # weights: a frame with weight 0 drops out
    w2 = np.array([[1.0, 0.0, 1.0]])
    H2 = pp.scharmer_raw(D, S, w2, [0], eta)
    ref2 = 1.0 - eta / (np.abs(O) ** 2 * (np.abs(S[0, 0]) ** 2 + np.abs(S[0, 2]) ** 2))
    np.testing.assert_allclose(H2, ref2, rtol=1e-12)


def test_scharmer_clip_median_island():
    """eta = 0 leaves H = 1 where the cross spectrum is nonzero; the final
    filter keeps only the part 4-connected to the origin after the median."""
    N = 16
    S = np.zeros((1, 1, N, N), complex)
    around = np.arange(-2, 3) % N
    S[0, 0][np.ix_(around, around)] = 1.0     # a 5x5 block centred on the origin
    S[0, 0, 8:11, 8:11] = 1.0                 # a detached 3x3 island
    D = S.copy()
    H = pp.scharmer_filter(D, S, np.ones((1, 1)), [0], 0.0)
    assert np.all(H[8:11, 8:11] == 0.0)
    assert H[0, 0] == 1.0 and H[1, 1] == 1.0 and H[2, 2] == 0.0   # corner loses the median
    ref = ndimage.median_filter(np.abs(S[0, 0]), 3, mode="wrap")
    ref[8:11, 8:11] = 0.0
    np.testing.assert_array_equal(H, ref)


def test_mosaic_reassembles_cut_patches():
    rng = np.random.default_rng(4)
    N, stride, ny, nx = 16, 8, 3, 4
    img = rng.standard_normal(((ny - 1) * stride + N, (nx - 1) * stride + N))
    patches = np.stack([img[i * stride:i * stride + N, k * stride:k * stride + N]
                        for i in range(ny) for k in range(nx)])
    for b in (0, 3, 6):
        np.testing.assert_allclose(pp.mosaic(patches, ny, nx, stride, b), img, atol=1e-13)
    const = np.full_like(patches, 2.5)
    np.testing.assert_allclose(pp.mosaic(const, ny, nx, stride, 4), 2.5, atol=1e-14)


def test_mosaic_weights_closed_form():
    """Two patches overlapping by half: the value at a pixel is the weighted
    mean of the two patch values with the taper weights."""
    N, b = 8, 3
    w = pp.taper(N, b)
    assert w[0, 0] == pytest.approx((0.5 * (1 - np.cos(np.pi * 0.5 / b))) ** 2)
    assert w[3, 3] == 1.0
    p = np.stack([np.full((N, N), 1.0), np.full((N, N), 3.0)])
    m = pp.mosaic(p, 1, 2, 4, b)
    y, x = 2, 5                                  # covered by both: x-x0 = 5 and 1
    ref = (w[y, 5] * 1.0 + w[y, 1] * 3.0) / (w[y, 5] + w[y, 1])
    assert m[y, x] == pytest.approx(ref, abs=1e-15)


def test_sector_masks_match_angles_and_radii():
    L = 64
    k, sector = pp.sector_masks(L)
    u = np.arange(L)
    u = np.where(u > L // 2, u - L, u)
    uy, ux = np.meshgrid(u, u, indexing="ij")
    r = np.hypot(ux, uy)
    np.testing.assert_array_equal(k, np.floor(r + 0.5).astype(int))
    ang = np.degrees(np.arctan2(np.abs(uy), np.abs(ux)))
    ref = (ux != 0) & (uy != 0) & (ang >= 30.0 - 1e-9) & (ang <= 60.0 + 1e-9)
    np.testing.assert_array_equal(sector, ref)
    assert sector[5, 5] and sector[-5, 5] and not sector[0, 7] and not sector[7, 1]


def test_power_spectrum_parseval_and_diagonal_wave():
    L = 32
    rng = np.random.default_rng(8)
    x = rng.standard_normal((L, L))
    P = pp.power_spectrum(x)
    assert P[0, 0] < 1e-20
    np.testing.assert_allclose(P.sum(), L * L * np.sum((x - x.mean()) ** 2), rtol=1e-12)
    # a plane wave along the diagonal, frequency (5, 5): all power at |u| = 7.07 -> bin 7
    yy, xx = np.mgrid[0:L, 0:L]
    wave = np.cos(2 * np.pi * 5 * (xx + yy) / L)
    mean, cnt = pp.sector_spectrum(pp.power_spectrum(wave), L // 2 + 1)
    assert np.argmax(mean) == 7 and np.count_nonzero(mean > 1e-9) == 1
    # an axis-aligned wave lies outside the sectors
    mean2, _ = pp.sector_spectrum(pp.power_spectrum(np.cos(2 * np.pi * 6 * xx / L)), L // 2 + 1)
    assert np.all(mean2 < 1e-9)
