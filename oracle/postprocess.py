"""FP64 oracle of the object post-processing -- test infrastructure.

Fourier filters of the restored object (Sect. "Fourier filtering") and the
mosaic of restored patches (Sect. "Division in patches and apodization").
Plain NumPy on the full N x N frequency grid; no code shared with the GPU
library.

Readings (where the text leaves a choice):
  * Frequencies are DFT bins u = (u_y, u_x) taken in (-N/2, N/2], with
    |u| = sqrt(u_y^2 + u_x^2); "units of the diffraction limit" divide |u| by
    the diffraction-limit frequency f_d in bins (D/lambda in pupil pixels),
    a caller parameter.
  * Top-hat: H = 1 for f <= f_l, 0 for f >= f_u, and
    H = (1 + cos(pi (f - f_l)/(f_u - f_l)))/2 in between.
  * Loefdahl-Scharmer: the printed ratio has no noise term; the filter is
    read as H = 1 - eta sum_j w |S_j|^2 / |sum_j w D_j conj(S_j)|^2 over the
    channels of the object, eta the noise power of a data frame per
    frequency bin (the printed form is eta = 1).  Values below 0.2 are set to
    0, values above 1 to 1; then a 3 x 3 median on the periodic frequency
    grid; then every nonzero value not 4-connected (periodically) to the
    zero frequency is set to 0.  Where the numerator sum vanishes H = 0.
  * The loss and gradient use the unfiltered Wiener object; the filter acts
    on the restored object only.
  * Mosaic weight: the separable cosine taper of the apodization window,
    w1(x) = (1 - cos(pi (e + 1/2)/b))/2 for e = min(x, N-1-x) < b, else 1;
    the mosaic is sum_p w o_p / sum_p w over the patches covering a pixel.
"""

from __future__ import annotations

from collections import deque

import numpy as np

from .momfbd import dft2, idft2_un


def frequency_radius(N: int) -> np.ndarray:
    """|u| in bins on the full grid, u in (-N/2, N/2]."""
    u = np.arange(N)
    u = np.where(u > N // 2, u - N, u).astype(np.float64)
    return np.sqrt(u[:, None] ** 2 + u[None, :] ** 2)


def tophat_filter(N: int, f_lo: float, f_hi: float, diff_limit: float) -> np.ndarray:
    """Top-hat filter with a cosine transition (Sect. "Fourier filtering")."""
    f = frequency_radius(N) / diff_limit
    H = np.zeros((N, N))
    H[f <= f_lo] = 1.0
    mid = (f > f_lo) & (f < f_hi)
    H[mid] = 0.5 * (1.0 + np.cos(np.pi * (f[mid] - f_lo) / (f_hi - f_lo)))
    return H


def median3_periodic(x: np.ndarray) -> np.ndarray:
    """3 x 3 median with periodic wrap-around."""
    stack = [np.roll(np.roll(x, dy, 0), dx, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return np.sort(np.stack(stack), axis=0)[4]


def connected_to_origin(mask: np.ndarray) -> np.ndarray:
    """Cells of `mask` 4-connected (periodically) to (0, 0), by breadth-first search."""
    N0, N1 = mask.shape
    keep = np.zeros_like(mask, dtype=bool)
    if not mask[0, 0]:
        return keep
    q = deque([(0, 0)])
    keep[0, 0] = True
    while q:
        y, x = q.popleft()
        for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            v, u = (y + dy) % N0, (x + dx) % N1
            if mask[v, u] and not keep[v, u]:
                keep[v, u] = True
                q.append((v, u))
    return keep


def scharmer_raw(D: np.ndarray, S: np.ndarray, w: np.ndarray, chans, noise_power: float):
    """1 - eta sum w|S|^2 / |sum w D conj(S)|^2 before clipping (full grid).

    D, S: [C][J][N][N] full spectra; chans: the channels of the object."""
    num = np.zeros(D.shape[-2:], np.complex128)
    den = np.zeros(D.shape[-2:])
    for c in chans:
        for j in range(D.shape[1]):
            num += w[c, j] * D[c, j] * np.conj(S[c, j])
            den += w[c, j] * np.abs(S[c, j]) ** 2
    mag = np.abs(num) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        H = np.where(mag > 0, 1.0 - noise_power * den / np.where(mag > 0, mag, 1.0), 0.0)
    return H


def scharmer_filter(D, S, w, chans, noise_power: float) -> np.ndarray:
    """Loefdahl-Scharmer filter: clip, median, keep the zero-frequency island."""
    H = scharmer_raw(D, S, w, chans, noise_power)
    H = np.where(H < 0.2, 0.0, np.minimum(H, 1.0))
    H = median3_periodic(H)
    return np.where(connected_to_origin(H > 0), H, 0.0)


def filtered_object(O: np.ndarray, H: np.ndarray) -> np.ndarray:
    """Restored object in pixel units after the filter: Re IDFT_un(H O) / N^2."""
    N = O.shape[-1]
    return idft2_un(H * O).real / (N * N)


def taper(N: int, b: int) -> np.ndarray:
    """Separable cosine taper of width b (b = 0: flat)."""
    x = np.arange(N)
    e = np.minimum(x, N - 1 - x).astype(np.float64)
    w1 = np.where(e < b, 0.5 * (1.0 - np.cos(np.pi * (e + 0.5) / max(b, 1))), 1.0)
    return w1[:, None] * w1[None, :]


def mosaic(patches: np.ndarray, ny: int, nx: int, stride: int, border: int) -> np.ndarray:
    """Weighted average of patches [ny*nx][N][N] placed at (i stride, k stride)."""
    N = patches.shape[-1]
    H = (ny - 1) * stride + N
    W = (nx - 1) * stride + N
    acc = np.zeros((H, W))
    wsum = np.zeros((H, W))
    wt = taper(N, border)
    for i in range(ny):
        for k in range(nx):
            y0, x0 = i * stride, k * stride
            acc[y0:y0 + N, x0:x0 + N] += wt * patches[i * nx + k]
            wsum[y0:y0 + N, x0:x0 + N] += wt
    return acc / wsum



def power_spectrum(image: np.ndarray, window=None) -> np.ndarray:
    """|DFT(w (x - mean))|^2 of a square image (direct DFT, FP64)."""
    x = np.asarray(image, np.float64)
    w = np.ones_like(x) if window is None else np.asarray(window, np.float64)
    X = dft2(w * (x - x.mean()))
    return X.real ** 2 + X.imag ** 2


def sector_masks(L: int):
    """Radial bin k = round(|u|) and the +-45 degree sector flag on the full
    grid, u in (-L/2, L/2]; decided with integer arithmetic:
    (2k-1)^2 <= 4|u|^2 < (2k+1)^2, and 30..60 degrees from the axes as
    u_x^2 <= 3 u_y^2 and u_y^2 <= 3 u_x^2 (both nonzero)."""
    u = np.arange(L)
    u = np.where(u > L // 2, u - L, u).astype(np.int64)
    uy, ux = np.meshgrid(u, u, indexing="ij")
    r4 = 4 * (ux ** 2 + uy ** 2)
    k = np.zeros_like(r4)
    while True:
        up = r4 >= (2 * k + 1) ** 2
        if not up.any():
            break
        k = k + up
    sector = (ux != 0) & (uy != 0) & (ux ** 2 <= 3 * uy ** 2) & (uy ** 2 <= 3 * ux ** 2)
    return k, sector


def sector_spectrum(P: np.ndarray, nbins: int):
    """Mean of P over the +-45 degree sectors (30 degrees wide) in each
    radial bin k = 0..nbins-1 (Sect. "Results"); returns (mean, count)."""
    k, sector = sector_masks(P.shape[0])
    sel = sector & (k < nbins)
    s = np.bincount(k[sel], weights=P[sel], minlength=nbins)[:nbins]
    c = np.bincount(k[sel], minlength=nbins)[:nbins]
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.where(c > 0, s / np.maximum(c, 1), 0.0)
    return mean, c
