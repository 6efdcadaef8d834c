"""FP64 oracle of the MOMFBD loss, gradient and object -- test infrastructure.

Every transform is a direct DFT through explicit DFT matrices whose phase
(u*r mod N) is reduced in integers before cos/sin are evaluated in float64.
No FFT library is used.  Inputs are the same float32 arrays the GPU library
reads, promoted to float64.

Conventions (readings of the paper, listed with their reasons in the design
notes):
  * DFT(x)(u) = sum_r x(r) exp(-2 pi i u.r/N) (unnormalised); the inverse used
    for the pupil is IDFT_un(X)(r) = sum_u X(u) exp(+2 pi i u.r/N), i.e. the
    F^-1 of the PSF equation without the 1/N^2.
  * PSF s = kappa |IDFT_un(P)|^2 with the closed-form kappa = 1/(N^2 sum A^2),
    which makes sum_r s = 1 for every wavefront (unit integral, Sect.
    "Spatially variant convolution" and Sect. "PSF").
  * No fftshift anywhere: the PSF peak of a flat wavefront sits at pixel (0,0).
  * The loss is summed over the full N x N frequency grid with no
    normalisation (Eq. loss_momfbd).
  * "gamma" is the Wiener constant S_n/S_0 of Eq. object_optimization, a
    scalar or a per-frequency array per object; the frame weights gamma_kj of
    Eq. log_posterior are called w here.
"""

from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Direct DFT (no FFT library)
# ---------------------------------------------------------------------------

_MAT_CACHE: dict = {}


def _dft_matrix(N: int, sign: int) -> np.ndarray:
    """F[u, r] = exp(sign * 2 pi i (u r mod N) / N), float64 complex."""
    key = (N, sign)
    if key not in _MAT_CACHE:
        u = np.arange(N, dtype=np.int64)
        ur = np.outer(u, u) % N
        ang = (2.0 * np.pi / N) * ur.astype(np.float64)
        _MAT_CACHE[key] = np.cos(ang) + 1j * sign * np.sin(ang)
    return _MAT_CACHE[key]


def _apply2(x: np.ndarray, sign: int) -> np.ndarray:
    """F0 x F1^T over the last two axes of a stack, as two large matrix products
    (the stack is folded into the free dimension of each product)."""
    x = np.asarray(x, dtype=np.complex128)
    n0, n1 = x.shape[-2], x.shape[-1]
    F0 = _dft_matrix(n0, sign)
    F1 = _dft_matrix(n1, sign)
    lead = x.shape[:-2]
    y = (x.reshape(-1, n1) @ F1.T).reshape(lead + (n0, n1))          # along columns
    y = np.swapaxes(y, -1, -2).reshape(-1, n0) @ F0.T                 # along rows
    return np.ascontiguousarray(np.swapaxes(y.reshape(lead + (n1, n0)), -1, -2))


def dft2(x: np.ndarray) -> np.ndarray:
    """Unnormalised forward 2-D DFT over the last two axes."""
    return _apply2(x, -1)


def idft2_un(X: np.ndarray) -> np.ndarray:
    """Unnormalised inverse 2-D DFT (exp(+2 pi i u.r/N), no 1/N^2)."""
    return _apply2(X, +1)


def expand_half(Xh: np.ndarray, N: int) -> np.ndarray:
    """Full N x N spectrum from the half spectrum [..., N, N/2+1] of real data.

    Columns 0..N/2 are taken as given; column kx > N/2 is the conjugate of
    column N-kx at row (-ky mod N) (Hermitian symmetry of a real signal).
    """
    Xh = np.asarray(Xh, dtype=np.complex128)
    out = np.empty(Xh.shape[:-1] + (N,), dtype=np.complex128)
    h = N // 2
    out[..., : h + 1] = Xh
    ky_neg = (-np.arange(N)) % N
    for kx in range(h + 1, N):
        out[..., :, kx] = np.conj(Xh[..., ky_neg, N - kx])
    return out


# ---------------------------------------------------------------------------
# Wavefront -> pupil -> PSF -> OTF (Sect. "Wavefronts", Eq. wavefront,
# Eq. pupil_func)
# ---------------------------------------------------------------------------

def wavefront(alpha_j: np.ndarray, basis_c: np.ndarray, div_c: np.ndarray) -> np.ndarray:
    """phi = sum_m alpha_m Z_m + theta (Eq. wavefront plus the known diversity).

    ``basis_c`` already carries the lambda_0/lambda_c factor of Eq. wavefront.
    """
    a = np.asarray(alpha_j, np.float64)
    Z = np.asarray(basis_c, np.float64)
    return np.tensordot(a, Z, axes=(0, 0)) + np.asarray(div_c, np.float64)


def pupil_field(A: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Generalised pupil P = A exp(i phi)."""
    return np.asarray(A, np.float64) * np.exp(1j * phi)


def psf_field(P: np.ndarray) -> np.ndarray:
    """Complex amplitude p = IDFT_un(P) (the F^-1 of Eq. pupil_func)."""
    return idft2_un(P)


def psf_kappa(A: np.ndarray) -> float:
    A = np.asarray(A, np.float64)
    N = A.shape[-1]
    return 1.0 / (N * N * float(np.sum(A * A)))


def psf(A: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Unit-sum PSF s = kappa |IDFT_un(A e^{i phi})|^2 (Eq. pupil_func)."""
    p = psf_field(pupil_field(A, phi))
    return psf_kappa(A) * (p.real ** 2 + p.imag ** 2)


def otf(s: np.ndarray) -> np.ndarray:
    """S = DFT(s), full grid."""
    return dft2(s)


# ---------------------------------------------------------------------------
# Object estimate, loss and gradient (Eqs. object_optimization, loss_momfbd)
# ---------------------------------------------------------------------------

def _gamma_full(gamma, K: int, N: int) -> np.ndarray:
    g = np.asarray(gamma, np.float64)
    if g.ndim == 0:
        return np.full((K, N, N), float(g))
    if g.shape == (K, N, N // 2 + 1):
        return expand_half(g, N).real
    if g.shape == (K, N, N):
        return g
    raise ValueError("gamma must be scalar, [K][N][N/2+1] or [K][N][N]")


def smoothness_gamma(N: int, gamma0, lam) -> np.ndarray:
    """Per-frequency Wiener constant of the object smoothness prior.

    Sect. "Smoothness" (Eq. regularization_smoothness) penalises
    lambda_k ||grad o_k||^2.  With periodic forward differences
    (dx o)(r) = o(r + e_x) - o(r), Parseval turns the penalty into
    lambda_k / N^2 sum_u |O_k(u)|^2 |e^{2 pi i u_x/N} - 1|^2 + (same in y), and
    |e^{i t} - 1|^2 = 4 sin^2(t/2).  Scaling the pixel-domain objective by N^2
    (the unnormalised Fourier sum of Eq. loss_momfbd), a constant gamma0_k plus
    this penalty is the array gamma_k(u) = gamma0_k + lambda_k (4 sin^2(pi u_x/N)
    + 4 sin^2(pi u_y/N)) in the denominator of Eq. object_optimization.
    Returns float64 [K][N][N] on the full grid.
    """
    g0 = np.atleast_1d(np.asarray(gamma0, np.float64))
    lm = np.atleast_1d(np.asarray(lam, np.float64))
    u = np.arange(N)
    lap = 4.0 * np.sin(np.pi * u / N) ** 2
    grid = lap[:, None] + lap[None, :]
    return g0[:, None, None] + lm[:, None, None] * grid[None]


def accumulators(D: np.ndarray, S: np.ndarray, w: np.ndarray, chan_obj, gamma, K: int):
    """N_k = sum_{c in k, j} w D conj(S);  Q_k = sum w |S|^2 + gamma_k.

    D, S: full-grid spectra [C][J][N][N]; w: [C][J].  These are the numerator
    and denominator of the Wiener object of Eq. object_optimization.
    """
    C, J, N, _ = D.shape
    Nk = np.zeros((K, N, N), np.complex128)
    Qk = np.array(_gamma_full(gamma, K, N), copy=True)
    for c in range(C):
        k = int(chan_obj[c])
        for j in range(J):
            Nk[k] += w[c, j] * D[c, j] * np.conj(S[c, j])
            Qk[k] += w[c, j] * (S[c, j].real ** 2 + S[c, j].imag ** 2)
    return Nk, Qk


def loss_literal(D, S, w, chan_obj, gamma, K):
    """Eq. loss_momfbd as printed: sum_k,u [sum w|D|^2 - |sum w D^* S|^2 / Q]."""
    Nk, Qk = accumulators(D, S, w, chan_obj, gamma, K)
    C, J = D.shape[:2]
    total = 0.0
    for k in range(K):
        e = np.zeros(D.shape[-2:])
        for c in range(C):
            if int(chan_obj[c]) != k:
                continue
            for j in range(J):
                e += w[c, j] * np.abs(D[c, j]) ** 2
        total += float(np.sum(e - np.abs(Nk[k]) ** 2 / Qk[k]))
    return total


def evaluate_patch(alpha, D_half, basis, diversity, pupil, chan_obj, gamma,
                   weights=None, want_grad=True):
    """Loss, gradient and object of one patch.

    alpha [J][M]; D_half [C][J][N][N/2+1] complex; basis [C][M][N][N];
    diversity, pupil [C][N][N]; chan_obj [C]; gamma scalar or per object.

    Loss: the residual form sum_k sum_u [sum_{c in k,j} w |D - O S|^2
    + gamma |O|^2] with O = N/Q, equal to Eq. loss_momfbd at the optimum.
    Gradient: the object is held at its optimum (envelope theorem), then the
    chain D,O -> S -> s -> p -> P -> phi -> alpha is taken by hand:
      G = -2 w conj(O) R,  g_s = Re IDFT_un(G),  H = 2 kappa g_s p,
      G_P = DFT(H),  g_phi = Im(conj(P) G_P),  dL/dalpha_m = sum_c sum_v Z_cm g_phi.
    """
    alpha = np.asarray(alpha, np.float64)
    C = len(chan_obj)
    J, M = alpha.shape
    N = pupil.shape[-1]
    K = int(np.max(chan_obj)) + 1
    w = np.ones((C, J)) if weights is None else np.asarray(weights, np.float64)
    D = expand_half(D_half, N)
    S = np.empty((C, J, N, N), np.complex128)
    s_all = np.empty((C, J, N, N))
    p_all = np.empty((C, J, N, N), np.complex128)
    P_all = np.empty((C, J, N, N), np.complex128)
    kap = np.empty(C)
    for c in range(C):
        kap[c] = psf_kappa(pupil[c])
        for j in range(J):
            phi = wavefront(alpha[j], basis[c], diversity[c])
            P = pupil_field(pupil[c], phi)
            p = psf_field(P)
            s = kap[c] * (p.real ** 2 + p.imag ** 2)
            P_all[c, j], p_all[c, j], s_all[c, j] = P, p, s
            S[c, j] = otf(s)
    Nk, Qk = accumulators(D, S, w, chan_obj, gamma, K)
    O = Nk / Qk
    gam = _gamma_full(gamma, K, N)
    loss = 0.0
    R = np.empty_like(D)
    for k in range(K):
        loss += float(np.sum(gam[k] * np.abs(O[k]) ** 2))
    for c in range(C):
        k = int(chan_obj[c])
        for j in range(J):
            R[c, j] = D[c, j] - O[k] * S[c, j]
            loss += float(w[c, j] * np.sum(R[c, j].real ** 2 + R[c, j].imag ** 2))
    out = dict(loss=loss, O=O, S=S, s=s_all, N=Nk, Q=Qk)
    if want_grad:
        grad = np.zeros((J, M))
        for c in range(C):
            k = int(chan_obj[c])
            Zc = np.asarray(basis[c], np.float64).reshape(M, -1)
            for j in range(J):
                G = -2.0 * w[c, j] * np.conj(O[k]) * R[c, j]
                g_s = idft2_un(G).real
                H = 2.0 * kap[c] * g_s * p_all[c, j]
                GP = dft2(H)
                g_phi = (np.conj(P_all[c, j]) * GP).imag
                grad[j] += Zc @ g_phi.ravel()
        out["grad"] = grad
    return out


def evaluate(alpha, D_half, basis, diversity, pupil, chan_obj, gamma, weights=None,
             patches=None, want_grad=True):
    """evaluate_patch over patches (all, or the listed indices)."""
    P = alpha.shape[0]
    idx = range(P) if patches is None else patches
    res = [evaluate_patch(alpha[p], D_half[p], basis, diversity, pupil, chan_obj,
                          gamma, weights, want_grad) for p in idx]
    out = dict(loss=np.array([r["loss"] for r in res]),
               O=np.stack([r["O"] for r in res]))
    if want_grad:
        out["grad"] = np.stack([r["grad"] for r in res])
    return out


def object_image(O: np.ndarray) -> np.ndarray:
    """Restored object in pixel units: o = Re IDFT_un(O) / N^2."""
    N = O.shape[-1]
    return idft2_un(O).real / float(N * N)


# ---------------------------------------------------------------------------
# Data preparation and the generative model (Sect. "Division in patches and
# apodization", Eq. generative_model)
# ---------------------------------------------------------------------------

def patch_spectra(patches: np.ndarray, window: np.ndarray) -> np.ndarray:
    """D = DFT(W (x - m) + m), m the per-frame patch mean; half spectrum.

    ``patches`` [..., N, N] real; returns [..., N, N/2+1] complex128.
    """
    x = np.asarray(patches, np.float64)
    N = x.shape[-1]
    m = x.mean(axis=(-2, -1), keepdims=True)
    y = np.asarray(window, np.float64) * (x - m) + m
    return dft2(y)[..., : N // 2 + 1]


def prepare_data(frames: np.ndarray, window: np.ndarray, N: int, stride: int) -> np.ndarray:
    """Cut frames [C][J][H][W] into the patch grid and transform each patch.

    Patch corners are y0 = i*stride for i = 0..(H-N)//stride, likewise x0;
    patches are ordered row-major over (i_y, i_x).  Returns
    [P][C][J][N][N/2+1] complex128.
    """
    C, J, H, W = frames.shape
    ny = (H - N) // stride + 1
    nx = (W - N) // stride + 1
    out = []
    for iy in range(ny):
        for ix in range(nx):
            y0, x0 = iy * stride, ix * stride
            out.append(patch_spectra(frames[:, :, y0:y0 + N, x0:x0 + N], window))
    return np.stack(out)


def simulate_frames(objects, alpha, basis, diversity, pupil, chan_obj, noise=None):
    """Frames i_cj = o_k(c) (*) s_cj + n_cj, circular convolution per patch.

    objects [P][K][N][N]; alpha [P][J][M]; returns [P][C][J][N][N] float64.
    This is the isoplanatic generative model (Eq. generative_model with the
    convolution of Sect. "Spatially invariant convolution").
    """
    P, J, M = alpha.shape
    C = len(chan_obj)
    N = pupil.shape[-1]
    out = np.empty((P, C, J, N, N))
    Ok = dft2(objects)                                          # [P][K][N][N]
    a = np.asarray(alpha, np.float64)
    for c in range(C):
        # all patches and frames of the channel at once (stacked 2-D transforms)
        phi = np.tensordot(a, np.asarray(basis[c], np.float64), axes=(2, 0)) \
            + np.asarray(diversity[c], np.float64)              # [P][J][N][N]
        s = psf(pupil[c], phi)
        img = idft2_un(Ok[:, int(chan_obj[c])][:, None] * otf(s)).real / float(N * N)
        out[:, c] = img if noise is None else img + noise[:, c]
    return out
