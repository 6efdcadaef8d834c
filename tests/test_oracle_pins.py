"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, textbook special cases (Airy pattern, pupil autocorrelation), an
independent library routine (numpy.fft for the direct DFT), brute force on
tiny inputs (dense circulant least squares), invariances of the method
(tilt, even-mode sign flips) and central finite differences.
"""

import numpy as np
import pytest
from scipy.special import j1

import oracle
import synth


def _rng(k):
    return np.random.default_rng(1000 + k)


# ---------------------------------------------------------------- DFT -------

@pytest.mark.parametrize("N", [8, 16, 64])
def test_dft_matches_numpy_fft(N):
    x = _rng(N).standard_normal((N, N)) + 1j * _rng(N + 1).standard_normal((N, N))
    np.testing.assert_allclose(oracle.dft2(x), np.fft.fft2(x), rtol=0, atol=1e-10 * N * N)
    np.testing.assert_allclose(oracle.idft2_un(x), np.fft.ifft2(x) * N * N, rtol=0,
                               atol=1e-10 * N * N)


def test_dft_closed_forms():
    N = 64
    delta = np.zeros((N, N))
    delta[0, 0] = 1.0
    np.testing.assert_allclose(oracle.dft2(delta), np.ones((N, N)), atol=1e-13)
    const = np.full((N, N), 3.0)
    X = oracle.dft2(const)
    assert abs(X[0, 0] - 3.0 * N * N) < 1e-9
    X[0, 0] = 0
    assert np.max(np.abs(X)) < 1e-10
    # single cosine along x at frequency 5: two bins of N^2/2
    r = np.arange(N)
    cosx = np.tile(np.cos(2 * np.pi * 5 * r / N), (N, 1))
    X = oracle.dft2(cosx)
    assert abs(X[0, 5] - N * N / 2) < 1e-9 and abs(X[0, N - 5] - N * N / 2) < 1e-9
    X[0, 5] = X[0, N - 5] = 0
    assert np.max(np.abs(X)) < 1e-9


def test_parseval_and_inverse():
    N = 64
    x = _rng(3).standard_normal((N, N))
    X = oracle.dft2(x)
    assert abs(np.sum(np.abs(X) ** 2) - N * N * np.sum(x ** 2)) < 1e-9 * N * N * np.sum(x ** 2)
    np.testing.assert_allclose(oracle.idft2_un(X).real, N * N * x, atol=1e-9)


def test_expand_half_matches_full_spectrum():
    N = 16
    x = _rng(4).standard_normal((3, N, N))
    full = np.fft.fft2(x)
    np.testing.assert_allclose(oracle.expand_half(full[..., : N // 2 + 1], N), full, atol=1e-12)


# ------------------------------------------------------- generator -------

def test_noll_indices():
    expect = {1: (0, 0), 2: (1, 1), 3: (1, -1), 4: (2, 0), 5: (2, -2), 6: (2, 2),
              7: (3, -1), 8: (3, 1), 9: (3, -3), 10: (3, 3), 11: (4, 0), 12: (4, 2),
              13: (4, -2), 22: (6, 0)}
    for j, nm in expect.items():
        assert synth.noll_to_nm(j) == nm


def test_zernike_tilts_are_linear_and_near_orthonormal():
    N = 64
    R = synth.pupil_radius_px(N)
    Z = synth.zernike_basis(N, 44)
    A = synth.pupil_mask(N)
    v = np.arange(N) - N // 2
    vy, vx = np.meshgrid(v, v, indexing="ij")
    np.testing.assert_allclose(Z[0], np.where(A > 0, 2 * vx / R, 0), atol=1e-12)
    np.testing.assert_allclose(Z[1], np.where(A > 0, 2 * vy / R, 0), atol=1e-12)
    G = (Z.reshape(44, -1) @ Z.reshape(44, -1).T) / A.sum()
    # pixelated 657-pixel disc: low orders are orthonormal to ~4e-2,
    # the highest orders here to ~0.1 (a missing sqrt(2) would give 0.5)
    assert np.max(np.abs(G[:10, :10] - np.eye(10))) < 0.05
    assert np.max(np.abs(G - np.eye(44))) < 0.15


def test_noll_covariance_matches_noll_table():
    rows = [l.split() for l in open(__file__.replace("test_oracle_pins.py",
                                                     "golden/noll1976_residuals.txt"))
            if l.strip() and not l.startswith("#")]
    delta = {int(a): float(b) for a, b in rows}
    cov = synth.noll_covariance(20)
    for j in range(2, 22):
        var_tab = delta[j - 1] - delta[j]
        tol = 6e-4 if j <= 5 else 1e-4      # Delta_1..4 carry 3 decimals, the rest 4
        assert abs(cov[j - 2, j - 2] - var_tab) < tol, j
    # tilt-coma correlation of Noll's paper: <a2 a8> = -0.0141 (D/r0)^5/3
    assert abs(cov[0, 6] + 0.0141) < 2e-4


def test_kolmogorov_draw_statistics():
    rng = np.random.default_rng(5)
    a = synth.draw_kolmogorov(rng, 20000, 20, 10.0, ao_modes=0)
    target = synth.noll_covariance(20, 10.0)
    var = a.var(axis=0)
    rel = np.abs(var / np.diag(target) - 1)
    assert np.all(rel < 5 * np.sqrt(2 / 20000)), rel.max()
    a2 = synth.draw_kolmogorov(rng, 20000, 20, 10.0)
    np.testing.assert_allclose(a2[:, :9].std(0) / a[:, :9].std(0), 0.3, rtol=0.05)


def test_object_field_statistics():
    rng = np.random.default_rng(6)
    o = synth.object_field(rng, 512)
    assert abs(o.mean() - 1.0) < 2e-3 and abs(o.std() - 0.1) < 2e-3
    P = np.abs(np.fft.fft2(o - o.mean())) ** 2
    k = np.hypot(*np.meshgrid(np.fft.fftfreq(512), np.fft.fftfreq(512), indexing="ij"))
    bins = np.logspace(np.log10(0.01), np.log10(0.3), 12)
    kc, pc = [], []
    for lo, hi in zip(bins[:-1], bins[1:]):
        m = (k >= lo) & (k < hi)
        kc.append(np.sqrt(lo * hi))
        pc.append(P[m].mean())
    slope = np.polyfit(np.log(kc), np.log(pc), 1)[0]
    assert abs(slope + 3.0) < 0.1, slope


def test_hann_window():
    w = synth.hann_window(64, 6)
    assert w[32, 32] == 1.0 and w[0, 32] < 0.02 and np.allclose(w, w[::-1, ::-1])
    e = np.arange(6)
    np.testing.assert_allclose(w[32, :6], 0.5 * (1 - np.cos(np.pi * (e + 0.5) / 6)))


# -------------------------------------------------------- PSF / OTF -------

def test_psf_unit_sum_nonnegative_strehl():
    pr = synth.make_problem(11, P=1, J=4, M=44, d_over_r0=15.0)
    A = pr.pupil[0].astype(np.float64)
    peak0 = oracle.psf(A, np.zeros((64, 64))).max()
    assert peak0 == A.sum() / 64 ** 2          # 657/4096, exact in binary
    assert peak0 == 0.160400390625
    for j in range(4):
        phi = oracle.wavefront(pr.alpha_true[0, j], pr.basis[0], pr.diversity[0])
        s = oracle.psf(A, phi)
        assert abs(s.sum() - 1.0) < 1e-13
        assert s.min() >= 0.0 and s.max() <= peak0 * (1 + 1e-12)


@pytest.mark.parametrize("N,tol", [(64, 1.5e-3), (128, 4e-4)])
def test_flat_wavefront_psf_is_airy(N, tol):
    """A flat wavefront gives the Airy pattern of the disc with the same area
    as the pixelated aperture (the residual is the pixelation of the disc)."""
    A = synth.pupil_mask(N)
    s = oracle.psf(A, np.zeros((N, N)))
    d = 2.0 * np.sqrt(A.sum() / np.pi)
    r = np.minimum(np.arange(N), N - np.arange(N))
    ry, rx = np.meshgrid(r, r, indexing="ij")
    x = np.pi * d * np.hypot(ry, rx) / N
    airy = np.ones_like(x)
    nz = x > 0
    airy[nz] = (2 * j1(x[nz]) / x[nz]) ** 2
    airy *= A.sum() / N ** 2
    assert np.max(np.abs(s - airy)) / s.max() <= tol


def _autocorr_otf(P):
    """S(u) = sum_v conj(P(v)) P(v+u) / sum |A|^2, by direct circular sums."""
    N = P.shape[0]
    norm = np.sum(np.abs(P) ** 2)
    out = np.empty((N, N), complex)
    for uy in range(N):
        for ux in range(N):
            out[uy, ux] = np.sum(np.conj(P) * np.roll(P, (-uy, -ux), axis=(0, 1)))
    return out / norm


def test_otf_is_pupil_autocorrelation():
    N = 32
    A = synth.pupil_mask(N)
    Z = synth.zernike_basis(N, 10)
    phi = np.tensordot(_rng(8).standard_normal(10), Z, 1)
    P = oracle.pupil_field(A, phi)
    S = oracle.otf(oracle.psf(A, phi))
    np.testing.assert_allclose(S, _autocorr_otf(P), atol=1e-12)
    # Hermitian, unit DC, band limit |u| <= d
    assert abs(S[0, 0] - 1) < 1e-13
    np.testing.assert_allclose(S[(-np.arange(N)) % N][:, (-np.arange(N)) % N], np.conj(S),
                               atol=1e-13)
    r = np.minimum(np.arange(N), N - np.arange(N))
    u = np.hypot(*np.meshgrid(r, r, indexing="ij"))
    assert np.max(np.abs(S[u > 0.45 * N + 1])) < 1e-12


def test_flat_otf_is_overlap_count():
    N = 64
    A = synth.pupil_mask(N)
    S = oracle.otf(oracle.psf(A, np.zeros((N, N))))
    cnt = np.empty((N, N))
    for uy in range(N):
        for ux in range(N):
            cnt[uy, ux] = np.sum(A * np.roll(A, (-uy, -ux), axis=(0, 1)))
    np.testing.assert_allclose(S.real, cnt / A.sum(), atol=1e-12)
    assert np.max(np.abs(S.imag)) < 1e-12
    assert int(np.sum(cnt > 0)) == 2577


# ----------------------------------------------- loss / object / grad -------

def _small_problem(N=16, J=3, M=6, C=1, seed=21, noise=0.01, diversity=False):
    chans = ((0, 0.0),) if C == 1 else ((0, 0.0), (0, 1.0 if diversity else 0.0))
    pr = synth.make_problem(seed, N=N, P=1, J=J, M=M, channels=chans, d_over_r0=6.0,
                            border=2, noise_sigma=noise)
    frames = oracle.simulate_frames(pr.objects, pr.alpha_true, pr.basis, pr.diversity,
                                    pr.pupil, pr.channel_object, pr.noise)
    D = oracle.patch_spectra(frames, pr.window)
    return pr, D


def test_residual_form_equals_literal_loss():
    pr, D = _small_problem(N=64, J=5, M=20, C=2, diversity=True)
    a = pr.alpha_true[0] + 0.3 * _rng(9).standard_normal(pr.alpha_true[0].shape)
    r = oracle.evaluate_patch(a, D[0], pr.basis, pr.diversity, pr.pupil,
                              pr.channel_object, pr.gamma, want_grad=False)
    lit = oracle.loss_literal(oracle.expand_half(D[0], 64), r["S"], np.ones((2, 5)),
                              pr.channel_object, pr.gamma, 1)
    assert abs(r["loss"] - lit) <= 1e-12 * abs(lit)


def _circulant(s):
    """Dense matrix C with (C o)(r) = sum_r' s(r - r') o(r') on the N x N torus."""
    N = s.shape[0]
    n = N * N
    Cm = np.empty((n, n))
    for ry in range(N):
        for rx in range(N):
            Cm[ry * N + rx] = np.roll(np.roll(s[::-1, ::-1], ry + 1, 0), rx + 1, 1).ravel()
    return Cm


def _psf_direct(A, phi):
    """|sum_v P(v) exp(+2 pi i v.r/N)|^2 / (N^2 sum A^2) by explicit sums."""
    N = A.shape[0]
    P = A * np.exp(1j * phi)
    v = np.arange(N)
    s = np.empty((N, N))
    for ry in range(N):
        for rx in range(N):
            ph = np.exp(2j * np.pi * (np.outer(v, np.ones(N)) * ry + np.outer(np.ones(N), v) * rx) / N)
            s[ry, rx] = abs(np.sum(P * ph)) ** 2
    return s / (N * N * np.sum(A * A))


def test_loss_equals_dense_real_space_least_squares():
    N, J, M = 8, 3, 5
    pr, _ = _small_problem(N=N, J=J, M=M)
    rng = _rng(10)
    frames = rng.standard_normal((J, N, N)) + 1.0
    D = oracle.dft2(frames)[:, :, : N // 2 + 1]
    a = pr.alpha_true[0].astype(np.float64)
    w = np.array([1.0, 0.5, 2.0])
    gam = 0.03
    r = oracle.evaluate_patch(a, D[None], pr.basis, pr.diversity, pr.pupil,
                              pr.channel_object, gam, w[None], want_grad=False)
    # independent: PSFs by explicit sums, object by dense normal equations
    A = pr.pupil[0].astype(np.float64)
    Cs = [_circulant(_psf_direct(A, oracle.wavefront(a[j], pr.basis[0], pr.diversity[0])))
          for j in range(J)]
    n = N * N
    lhs = gam * np.eye(n) + sum(w[j] * Cs[j].T @ Cs[j] for j in range(J))
    rhs = sum(w[j] * Cs[j].T @ frames[j].ravel() for j in range(J))
    o = np.linalg.solve(lhs, rhs)
    brute = sum(w[j] * np.sum((frames[j].ravel() - Cs[j] @ o) ** 2) for j in range(J))
    brute += gam * np.sum(o ** 2)
    assert abs(r["loss"] - n * brute) <= 1e-11 * abs(r["loss"])
    np.testing.assert_allclose(oracle.object_image(r["O"][0]), o.reshape(N, N), atol=1e-11)


def _forward_difference(N, axis):
    """Dense matrix of the periodic forward difference o(r + e_axis) - o(r)."""
    n = N * N
    G = -np.eye(n)
    for ry in range(N):
        for rx in range(N):
            ty, tx = ((ry + 1) % N, rx) if axis == 0 else (ry, (rx + 1) % N)
            G[ry * N + rx, ty * N + tx] += 1.0
    return G


def test_smoothness_gamma_equals_pixel_gradient_penalty():
    """The per-frequency gamma of the smoothness prior gives N^2 times the
    minimum of sum_j w ||d_j - o * s_j||^2 + gamma0 ||o||^2 + lambda ||grad o||^2
    over real objects, with the gradient as explicit periodic differences."""
    N, J, M = 8, 3, 5
    pr, _ = _small_problem(N=N, J=J, M=M)
    rng = _rng(11)
    frames = rng.standard_normal((J, N, N)) + 1.0
    D = oracle.dft2(frames)[:, :, : N // 2 + 1]
    a = pr.alpha_true[0].astype(np.float64)
    w = np.array([1.0, 0.5, 2.0])
    gam0, lam = 0.01, 0.3
    gam = oracle.smoothness_gamma(N, [gam0], [lam])
    r = oracle.evaluate_patch(a, D[None], pr.basis, pr.diversity, pr.pupil,
                              pr.channel_object, gam, w[None], want_grad=False)
    A = pr.pupil[0].astype(np.float64)
    Cs = [_circulant(_psf_direct(A, oracle.wavefront(a[j], pr.basis[0], pr.diversity[0])))
          for j in range(J)]
    Gy, Gx = _forward_difference(N, 0), _forward_difference(N, 1)
    n = N * N
    lhs = (gam0 * np.eye(n) + lam * (Gy.T @ Gy + Gx.T @ Gx)
           + sum(w[j] * Cs[j].T @ Cs[j] for j in range(J)))
    rhs = sum(w[j] * Cs[j].T @ frames[j].ravel() for j in range(J))
    o = np.linalg.solve(lhs, rhs)
    brute = sum(w[j] * np.sum((frames[j].ravel() - Cs[j] @ o) ** 2) for j in range(J))
    brute += gam0 * np.sum(o ** 2) + lam * (np.sum((Gy @ o) ** 2) + np.sum((Gx @ o) ** 2))
    assert abs(r["loss"] - n * brute) <= 1e-11 * abs(r["loss"])
    np.testing.assert_allclose(oracle.object_image(r["O"][0]), o.reshape(N, N), atol=1e-11)
    # lambda = 0 reduces to the constant gamma; the table is symmetric in u -> -u
    np.testing.assert_array_equal(oracle.smoothness_gamma(N, [gam0], [0.0])[0], np.full((N, N), gam0))
    g = gam[0]
    np.testing.assert_allclose(g, np.roll(g[::-1, ::-1], 1, (0, 1)), atol=1e-15)


def test_noise_free_object_recovers_band_limited_truth():
    N, J = 64, 6
    pr = synth.make_problem(12, N=N, P=1, J=J, M=20, d_over_r0=8.0, noise_sigma=0.0)
    frames = oracle.simulate_frames(pr.objects, pr.alpha_true, pr.basis, pr.diversity,
                                    pr.pupil, pr.channel_object, None)
    D = oracle.patch_spectra(frames, np.ones((N, N)))
    r = oracle.evaluate_patch(pr.alpha_true[0], D[0], pr.basis, pr.diversity, pr.pupil,
                              pr.channel_object, 1e-14, want_grad=False)
    A = pr.pupil[0].astype(np.float64)
    support = np.abs(oracle.otf(oracle.psf(A, np.zeros((N, N))))) > 1e-9
    truth_bl = oracle.object_image(oracle.dft2(pr.objects[0, 0]) * support)
    err = oracle.object_image(r["O"][0]) - truth_bl
    assert np.sqrt(np.mean(err ** 2)) < 1e-8
    assert r["loss"] < 1e-12 * np.sum(np.abs(D) ** 2)


def test_gradient_central_differences():
    pr, D = _small_problem(N=32, J=3, M=8, C=2, diversity=True)
    a = pr.alpha_true[0].astype(np.float64) + 0.2 * _rng(13).standard_normal((3, 8))
    args = (D[0], pr.basis, pr.diversity, pr.pupil, pr.channel_object, 1e-2)
    g = oracle.evaluate_patch(a, *args)["grad"]
    h = 1e-6
    fd = np.empty_like(g)
    for j in range(3):
        for m in range(8):
            ap, am = a.copy(), a.copy()
            ap[j, m] += h
            am[j, m] -= h
            fd[j, m] = (oracle.evaluate_patch(ap, *args, want_grad=False)["loss"]
                        - oracle.evaluate_patch(am, *args, want_grad=False)["loss"]) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)


def test_common_tilt_and_even_flip_invariances():
    pr, D = _small_problem(N=64, J=4, M=20)
    a = pr.alpha_true[0].astype(np.float64)
    # float64 basis: the tilt modes must be exactly linear for exact invariance
    Z64 = synth.zernike_basis(64, 20)[None]
    args = (D[0], Z64, pr.diversity, pr.pupil, pr.channel_object, pr.gamma)
    r0 = oracle.evaluate_patch(a, *args)
    g = r0["grad"]
    # a common tilt shifts every PSF alike: no change of the loss, zero summed gradient
    assert abs(g[:, 0].sum()) < 1e-9 * np.abs(g).max()
    assert abs(g[:, 1].sum()) < 1e-9 * np.abs(g).max()
    at = a.copy()
    at[:, 0] += 0.37
    at[:, 1] -= 1.21
    assert abs(oracle.evaluate_patch(at, *args, want_grad=False)["loss"] - r0["loss"]) \
        < 1e-11 * r0["loss"]
    # flipping the sign of all even (even radial order) modes of one frame keeps its PSF
    even = np.array([synth.noll_to_nm(j + 2)[0] % 2 == 0 for j in range(20)])
    F = np.ones((4, 20))
    F[1, even] = -1.0
    F[3, even] = -1.0
    r1 = oracle.evaluate_patch(a * F, *args)
    assert abs(r1["loss"] - r0["loss"]) < 1e-11 * r0["loss"]
    np.testing.assert_allclose(r1["grad"], F * g, atol=1e-9 * np.abs(g).max())


def test_two_objects_decompose_into_single_object_problems():
    """Objects share no accumulator (Eq. object_optimization is per object):
    with two objects, each seen through its own channel, the loss and the
    gradient (the coefficients are shared) are the sums of those of the two
    one-object problems.  Pins the channel-to-object map: summing the
    channels of object 1 into object 0's N and Q, or the other way round,
    changes both."""
    N, J, M = 32, 3, 8
    pr = synth.make_problem(27, N=N, P=1, J=J, M=M, channels=((0, 0.0), (1, 1.0), (1, 0.0)),
                            d_over_r0=7.0, border=3)
    frames = oracle.simulate_frames(pr.objects, pr.alpha_true, pr.basis, pr.diversity,
                                    pr.pupil, pr.channel_object, pr.noise)
    D = oracle.patch_spectra(frames, pr.window)[0]
    a = pr.alpha_true[0].astype(np.float64) + 0.25 * _rng(27).standard_normal((J, M))
    w = np.array([[1.0, 0.6, 1.7], [0.8, 1.2, 0.5], [1.4, 0.9, 1.1]])
    gam = np.stack([np.full((N, N), 2e-3), np.full((N, N), 7e-3)])
    both = oracle.evaluate_patch(a, D, pr.basis, pr.diversity, pr.pupil, pr.channel_object,
                                 gam, w)
    parts = []
    for k, chans in ((0, [0]), (1, [1, 2])):
        parts.append(oracle.evaluate_patch(a, D[chans], pr.basis[chans], pr.diversity[chans],
                                           pr.pupil[chans], np.zeros(len(chans), np.int32),
                                           gam[k:k + 1], w[chans]))
    assert abs(both["loss"] - parts[0]["loss"] - parts[1]["loss"]) <= 1e-12 * both["loss"]
    np.testing.assert_allclose(both["grad"], parts[0]["grad"] + parts[1]["grad"], rtol=0,
                               atol=1e-11 * np.abs(both["grad"]).max())
    np.testing.assert_allclose(both["O"][1], parts[1]["O"][0], rtol=0,
                               atol=1e-12 * np.abs(both["O"][1]).max())
    # the pooled reading (every channel in one object) is a different problem
    pooled = oracle.evaluate_patch(a, D, pr.basis, pr.diversity, pr.pupil,
                                   np.zeros(3, np.int32), gam[:1], w)
    assert abs(pooled["loss"] - both["loss"]) > 1e-3 * both["loss"]


def test_diversity_is_a_known_coefficient_offset():
    """Eq. wavefront adds the diversity theta_c to the modal sum, so a
    diversity that is itself a modal sum Z beta gives the loss and gradient
    of the coefficients alpha + beta without diversity.  Pins the presence and
    the sign of the diversity term (dropping it or flipping it moves the
    loss by far more than rounding)."""
    N, J, M = 32, 3, 8
    pr, D = _small_problem(N=N, J=J, M=M, C=2, diversity=False)
    a = pr.alpha_true[0].astype(np.float64)
    Z = pr.basis.astype(np.float64)
    beta = np.array([0.4, -0.7, 0.9, 0.0, 0.3, -0.2, 0.5, -0.6])
    theta = np.stack([np.tensordot(beta, Z[c], axes=(0, 0)) for c in range(2)])
    theta[1] *= 0.5                     # a different offset per channel
    # channel c sees alpha + s_c beta; both channels share alpha, so compare
    # one channel at a time against its own shifted problem
    for c, sc in ((0, 1.0), (1, 0.5)):
        one = oracle.evaluate_patch(a, D[0][[c]], Z[[c]], theta[[c]], pr.pupil[[c]],
                                    np.zeros(1, np.int32), pr.gamma)
        shifted = oracle.evaluate_patch(a + sc * beta[None, :], D[0][[c]], Z[[c]],
                                        np.zeros((1, N, N)), pr.pupil[[c]],
                                        np.zeros(1, np.int32), pr.gamma)
        assert abs(one["loss"] - shifted["loss"]) <= 1e-12 * shifted["loss"]
        np.testing.assert_allclose(one["grad"], shifted["grad"], rtol=0,
                                   atol=1e-11 * np.abs(shifted["grad"]).max())
        flipped = oracle.evaluate_patch(a - sc * beta[None, :], D[0][[c]], Z[[c]],
                                        np.zeros((1, N, N)), pr.pupil[[c]],
                                        np.zeros(1, np.int32), pr.gamma)
        plain = oracle.evaluate_patch(a, D[0][[c]], Z[[c]], np.zeros((1, N, N)),
                                      pr.pupil[[c]], np.zeros(1, np.int32), pr.gamma)
        assert abs(flipped["loss"] - one["loss"]) > 1e-3 * one["loss"]
        assert abs(plain["loss"] - one["loss"]) > 1e-3 * one["loss"]
    # with one object fed by both channels the same holds for the shared alpha
    # when both channels are offset alike
    theta_same = np.stack([theta[0], theta[0]])
    both = oracle.evaluate_patch(a, D[0], Z, theta_same, pr.pupil, pr.channel_object, pr.gamma)
    ref = oracle.evaluate_patch(a + beta[None, :], D[0], Z, np.zeros((2, N, N)), pr.pupil,
                                pr.channel_object, pr.gamma)
    assert abs(both["loss"] - ref["loss"]) <= 1e-12 * ref["loss"]
    np.testing.assert_allclose(both["grad"], ref["grad"], rtol=0,
                               atol=1e-11 * np.abs(ref["grad"]).max())


# --------------------------------------------------- data preparation -------

def test_prepare_data_grid_and_transform():
    rng = _rng(14)
    C, J, H, W, N, stride = 2, 3, 40, 56, 16, 12
    frames = rng.standard_normal((C, J, H, W)) + 2.0
    win = synth.hann_window(N, 3)
    D = oracle.prepare_data(frames, win, N, stride)
    ny, nx = (H - N) // stride + 1, (W - N) // stride + 1
    assert D.shape == (ny * nx, C, J, N, N // 2 + 1)
    p = 1 * nx + 2                                        # patch (iy=1, ix=2)
    x = frames[1, 2, 12:28, 24:40]
    m = x.mean()
    ref = np.fft.rfft2(win * (x - m) + m)
    np.testing.assert_allclose(D[p, 1, 2], ref, atol=1e-10)
    flat = oracle.patch_spectra(np.full((N, N), 5.0), win)
    assert abs(flat[0, 0] - 5.0 * N * N) < 1e-10
    flat[0, 0] = 0
    assert np.max(np.abs(flat)) < 1e-10


def test_simulated_frames_are_circular_convolutions():
    N = 8
    pr = synth.make_problem(15, N=N, P=1, J=2, M=4, d_over_r0=5.0, noise_sigma=0.0)
    fr = oracle.simulate_frames(pr.objects, pr.alpha_true, pr.basis, pr.diversity,
                                pr.pupil, pr.channel_object, None)
    A = pr.pupil[0].astype(np.float64)
    for j in range(2):
        s = _psf_direct(A, oracle.wavefront(pr.alpha_true[0, j], pr.basis[0], pr.diversity[0]))
        o = pr.objects[0, 0]
        ref = np.zeros((N, N))
        for ry in range(N):
            for rx in range(N):
                for qy in range(N):
                    for qx in range(N):
                        ref[ry, rx] += o[qy, qx] * s[(ry - qy) % N, (rx - qx) % N]
        np.testing.assert_allclose(fr[0, 0, j], ref, atol=1e-12)
