"""Kolmogorov statistics of Zernike coefficients (Noll 1976).

The paper draws random wavefronts with Kolmogorov turbulence (Sect. "PSF",
citing Roddier 1990); the covariance of Noll-normalised Zernike coefficients
used here is Noll's closed form:

  <a_j a_j'> = c0 (-1)^((n+n'-2|m|)/2) sqrt((n+1)(n'+1))
               Gamma((n+n'-5/3)/2)
             / [Gamma((n-n'+17/3)/2) Gamma((n'-n+17/3)/2) Gamma((n+n'+23/3)/2)]
             * (D/r0)^(5/3)

with c0 = 0.0072 pi^(8/3) Gamma(14/3), nonzero only when |m| = |m'| and the
two modes have the same azimuthal parity (both cos, both sin, or m = 0).
Units: radians of phase at the reference wavelength.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import gamma as _gamma

from .geometry import noll_to_nm

_C0 = 0.0072 * math.pi ** (8.0 / 3.0) * _gamma(14.0 / 3.0)


def noll_covariance(n_modes: int, d_over_r0: float = 1.0,
                    first_noll: int = 2) -> np.ndarray:
    """Covariance matrix [n_modes][n_modes] of Zernike coefficients."""
    cov = np.zeros((n_modes, n_modes))
    idx = [first_noll + i for i in range(n_modes)]
    nm = [noll_to_nm(j) for j in idx]
    for a, (ja, (na, ma)) in enumerate(zip(idx, nm)):
        for b, (jb, (nb, mb)) in enumerate(zip(idx, nm)):
            if abs(ma) != abs(mb):
                continue
            if ma != 0 and (ja - jb) % 2 != 0:
                continue
            sgn = (-1) ** ((na + nb - 2 * abs(ma)) // 2)
            cov[a, b] = (_C0 * sgn * math.sqrt((na + 1) * (nb + 1))
                         * _gamma((na + nb - 5.0 / 3.0) / 2.0)
                         / (_gamma((na - nb + 17.0 / 3.0) / 2.0)
                            * _gamma((nb - na + 17.0 / 3.0) / 2.0)
                            * _gamma((na + nb + 23.0 / 3.0) / 2.0)))
    return cov * d_over_r0 ** (5.0 / 3.0)


def draw_kolmogorov(rng: np.random.Generator, n_draws: int, n_modes: int,
                    d_over_r0, ao_modes: int = 9, ao_factor: float = 0.3,
                    first_noll: int = 2) -> np.ndarray:
    """Draw [n_draws][n_modes] coefficients with Noll's covariance.

    ``d_over_r0`` is a scalar or an array of length n_draws.  The first
    ``ao_modes`` modes (Noll 2..10 by default) are multiplied by
    ``ao_factor`` in amplitude, a crude model of partial AO correction.
    """
    L = np.linalg.cholesky(noll_covariance(n_modes, 1.0, first_noll))
    z = rng.standard_normal((n_draws, n_modes))
    a = z @ L.T
    scale = np.broadcast_to(np.asarray(d_over_r0, dtype=np.float64), (n_draws,))
    a *= (scale ** (5.0 / 6.0))[:, None]
    a[:, :ao_modes] *= ao_factor
    return a


def kl_transform(n_modes: int, first_noll: int = 2):
    """Karhunen-Loeve modes of Kolmogorov turbulence in the span of the first
    n_modes Zernikes (the paper's default basis, Sect. "Wavefronts": the
    diagonalisation of the Zernike covariance).

    Returns (U, var): KL_i = sum_j U[j, i] Z_j, ordered by decreasing
    variance var[i] (at D/r0 = 1).  Noll's covariance couples only modes of
    equal |m| and parity, so each such block is diagonalised on its own and
    a KL mode never mixes cos and sin terms.
    """
    cov = noll_covariance(n_modes, 1.0, first_noll)
    nm = [noll_to_nm(first_noll + i) for i in range(n_modes)]
    key = [(abs(m), 0 if m == 0 else (1 if m > 0 else -1)) for (_, m) in nm]
    U = np.zeros((n_modes, n_modes))
    var = np.zeros(n_modes)
    col = 0
    for k in sorted(set(key)):
        idx = [i for i in range(n_modes) if key[i] == k]
        w, v = np.linalg.eigh(cov[np.ix_(idx, idx)])
        for e in range(len(idx)):
            # sign: largest component positive, for a reproducible basis
            vec = v[:, e] * np.sign(v[np.argmax(np.abs(v[:, e])), e])
            U[idx, col] = vec
            var[col] = w[e]
            col += 1
    order = np.argsort(-var, kind="stable")
    return U[:, order], var[order]


def kl_basis(N: int, n_modes: int, diameter_frac: float = 0.45, scale: float = 1.0):
    """KL modes [n_modes][N][N] (radians per unit coefficient) and their
    variances at D/r0 = 1."""
    from .geometry import zernike_basis
    U, var = kl_transform(n_modes)
    Z = zernike_basis(N, n_modes, diameter_frac, scale=scale)
    return np.tensordot(U.T, Z, axes=1), var
