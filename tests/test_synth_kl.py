"""The Karhunen-Loeve basis of the input generator: orthogonal transform of
the Zernike span that diagonalises Noll's covariance, never mixing
azimuthal orders or parities; a wavefront is the same in either basis, so
the oracle's loss and gradient transform accordingly."""

import numpy as np

import oracle
import synth


def test_kl_transform_diagonalises_noll_covariance():
    M = 44
    U, var = synth.kl_transform(M)
    C = synth.noll_covariance(M)
    np.testing.assert_allclose(U.T @ U, np.eye(M), atol=1e-12)
    np.testing.assert_allclose(U.T @ C @ U, np.diag(var), atol=1e-14)
    assert np.all(np.diff(var) <= 1e-15) and np.all(var > 0)
    keys = [(abs(m), np.sign(m)) for (_, m) in (synth.noll_to_nm(j) for j in range(2, M + 2))]
    for i in range(M):
        used = {keys[j] for j in np.nonzero(np.abs(U[:, i]) > 1e-12)[0]}
        assert len(used) == 1
    # tilts: the two largest variances, equal (x and y), slightly above Noll's 0.448
    assert abs(var[0] - var[1]) < 1e-15 and 0.448 < var[0] < 0.46


def test_kl_coefficients_are_uncorrelated():
    M, n = 20, 40000
    rng = np.random.default_rng(0)
    a = synth.draw_kolmogorov(rng, n, M, 1.0, ao_modes=0)
    U, var = synth.kl_transform(M)
    b = a @ U
    cov = b.T @ b / n
    off = cov - np.diag(np.diag(cov))
    assert np.max(np.abs(off) / np.sqrt(np.outer(var, var))) < 4.0 / np.sqrt(n) * 3
    np.testing.assert_allclose(np.diag(cov), var, rtol=0.05)


def test_same_wavefront_same_loss_in_either_basis():
    N, J, M = 32, 3, 14
    pr = synth.make_problem(21, N=N, P=1, J=J, M=M, diameter_frac=0.45)
    U, _ = synth.kl_transform(M)
    Z = synth.zernike_basis(N, M, 0.45)
    KL, _ = synth.kl_basis(N, M, 0.45)
    a = pr.alpha_true[0].astype(np.float64)
    b = a @ U                                       # coefficients of the same wavefront
    np.testing.assert_allclose(np.tensordot(a, Z, axes=1), np.tensordot(b, KL, axes=1), atol=1e-12)
    rng = np.random.default_rng(1)
    D = oracle.dft2(rng.standard_normal((1, J, N, N)) + 1.0)[..., : N // 2 + 1]
    rz = oracle.evaluate_patch(a, D, Z[None], pr.diversity, pr.pupil, pr.channel_object, 1e-3)
    rk = oracle.evaluate_patch(b, D, KL[None], pr.diversity, pr.pupil, pr.channel_object, 1e-3)
    assert abs(rz["loss"] - rk["loss"]) <= 1e-11 * abs(rz["loss"])
    np.testing.assert_allclose(rk["grad"], rz["grad"] @ U, rtol=1e-9, atol=1e-9 * np.abs(rz["grad"]).max())
