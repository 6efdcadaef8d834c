"""Random object fields and detector noise.

The object is a stand-in for solar granulation: a periodic Gaussian random
field with isotropic power spectrum proportional to k^-3 (k in cycles/px,
DC removed), scaled to 10% rms contrast around a mean of 1 and clipped at
zero.  The spectral shaping uses numpy's FFT; it only makes test scenes.
"""

from __future__ import annotations

import numpy as np


def object_field(rng: np.random.Generator, H: int, W: int | None = None,
                 slope: float = -3.0, rms: float = 0.1,
                 mean: float = 1.0) -> np.ndarray:
    W = H if W is None else W
    white = rng.standard_normal((H, W))
    ky = np.fft.fftfreq(H)[:, None]
    kx = np.fft.fftfreq(W)[None, :]
    k = np.hypot(ky, kx)
    amp = np.zeros_like(k)
    amp[k > 0] = k[k > 0] ** (slope / 2.0)
    field = np.fft.ifft2(np.fft.fft2(white) * amp).real
    field -= field.mean()
    field *= rms / field.std()
    return np.clip(field + mean, 0.0, None)


def gaussian_noise(rng: np.random.Generator, shape, sigma: float) -> np.ndarray:
    return sigma * rng.standard_normal(shape)
