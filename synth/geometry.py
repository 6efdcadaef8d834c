"""Pupil-plane geometry: aperture mask, Zernike modes, diversity, window.

Conventions (the paper leaves them open; these are the readings used here):
  * The pupil grid has the same N x N size as the image patch.  The aperture
    is a binary disc A(v) = [|v - c| <= d/2] with an integer centre
    c = (N/2, N/2) and diameter d = 0.45 N pixels (the pupil sampling of the
    instrument table, Sect. "PSF"; d < N/2 keeps the OTF alias free).
  * Zernike modes follow Noll (1976): ordering, normalisation and the
    cos/sin convention (even j -> cos, odd j -> sin), evaluated at pixel
    centres with no discrete re-orthonormalisation.  Piston is excluded;
    modal index m = 0..M-1 maps to Noll j = m + 2 (Sect. "Wavefronts").
  * The apodization window is the paper's modified Hanning window (flat top,
    cosine border of b pixels; Sect. "Division in patches and apodization").
"""

from __future__ import annotations

import math

import numpy as np


def noll_to_nm(j: int) -> tuple[int, int]:
    """Radial order n and signed azimuthal order m of Noll index j >= 1.

    m > 0 marks the cosine mode, m < 0 the sine mode, m = 0 rotationally
    symmetric modes.
    """
    if j < 1:
        raise ValueError("Noll index starts at 1")
    n = 0
    rem = j - 1
    while rem > n:
        n += 1
        rem -= n
    # |m| takes the values of the same parity as n, in increasing order;
    # pairs (cos, sin) share one |m|.
    m_abs = (n % 2) + 2 * ((rem + ((n + 1) % 2)) // 2)
    if m_abs == 0:
        return n, 0
    return n, (m_abs if j % 2 == 0 else -m_abs)


def _radial(n: int, m_abs: int, rho: np.ndarray) -> np.ndarray:
    out = np.zeros_like(rho)
    for s in range((n - m_abs) // 2 + 1):
        c = ((-1) ** s * math.factorial(n - s)
             / (math.factorial(s) * math.factorial((n + m_abs) // 2 - s)
                * math.factorial((n - m_abs) // 2 - s)))
        out += c * rho ** (n - 2 * s)
    return out


def pupil_radius_px(N: int, diameter_frac: float = 0.45) -> float:
    return 0.5 * diameter_frac * N


def _polar(N: int, radius: float):
    c = N // 2
    v = np.arange(N, dtype=np.float64) - c
    vy, vx = np.meshgrid(v, v, indexing="ij")
    x = vx / radius
    y = vy / radius
    rho = np.hypot(x, y)
    theta = np.arctan2(y, x)
    return rho, theta


def pupil_mask(N: int, diameter_frac: float = 0.45) -> np.ndarray:
    """Binary circular aperture A(v) on the N x N pupil grid (float64)."""
    rho, _ = _polar(N, pupil_radius_px(N, diameter_frac))
    return (rho <= 1.0).astype(np.float64)


def zernike_basis(N: int, n_modes: int, diameter_frac: float = 0.45,
                  first_noll: int = 2, scale: float = 1.0) -> np.ndarray:
    """Noll-normalised Zernike modes j = first_noll .. first_noll+n_modes-1.

    Returns [n_modes][N][N] float64, zero outside the aperture, multiplied by
    ``scale`` (the wavelength factor lambda_0/lambda of the wavefront
    equation).
    """
    radius = pupil_radius_px(N, diameter_frac)
    rho, theta = _polar(N, radius)
    inside = rho <= 1.0
    out = np.zeros((n_modes, N, N))
    for i in range(n_modes):
        n, m = noll_to_nm(first_noll + i)
        r = _radial(n, abs(m), rho)
        if m == 0:
            z = math.sqrt(n + 1) * r
        elif m > 0:
            z = math.sqrt(2 * (n + 1)) * r * np.cos(m * theta)
        else:
            z = math.sqrt(2 * (n + 1)) * r * np.sin(-m * theta)
        out[i] = np.where(inside, z, 0.0) * scale
    return out


def defocus_diversity(N: int, waves_pv: float = 1.0,
                      diameter_frac: float = 0.45) -> np.ndarray:
    """Phase-diversity map for a defocus of ``waves_pv`` waves peak-to-valley.

    Defocus Z4 = sqrt(3)(2 rho^2 - 1) spans 2 sqrt(3) peak to valley, so one
    wave (2 pi rad) PV is (pi / sqrt 3) Z4 = pi (2 rho^2 - 1) rad.
    """
    z4 = zernike_basis(N, 1, diameter_frac, first_noll=4)[0]
    return waves_pv * (math.pi / math.sqrt(3.0)) * z4


def hann_window(N: int, border: int) -> np.ndarray:
    """Modified Hanning window: unity inside, cosine roll-off over ``border`` px.

    Separable; along one axis w(x) = (1 - cos(pi (e + 1/2) / b)) / 2 with
    e = min(x, N-1-x) when e < b, else 1.  border = N/2 gives a full Hann.
    """
    x = np.arange(N)
    e = np.minimum(x, N - 1 - x).astype(np.float64)
    w = np.where(e < border, 0.5 * (1.0 - np.cos(np.pi * (e + 0.5) / border)), 1.0)
    return np.outer(w, w)
