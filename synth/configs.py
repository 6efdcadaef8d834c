"""Seeded problem set-ups for the workloads the hot path is tested and timed on.

Everything is drawn from numpy.random.SeedSequence([SEED_ROOT, key]) spawned
into four streams: object, wavefront, noise, layout.

Workloads (all synthetic; the paper's observations are not available):
  * config0: one 64x64 patch, one object, 8 frames, 44 Zernike modes
    (Noll 2..45), Kolmogorov coefficients at D/r0 = 10 with modes 2..10
    scaled by 0.3, k^-3 object with 10% contrast, 1% Gaussian noise,
    gamma = 1e-3, modified Hanning window with a 6 px border.
  * config1: a 1024x1024 field cut into 64x64 patches at stride 32
    (31 x 31 = 961 patches), 12 frames, two objects (a wideband channel and a
    +1 wave peak-to-valley defocus phase-diversity channel) sharing the modal
    coefficients, 66 modes (Noll 2..67), D/r0 rising smoothly from 5 to 20
    across the field.
  * config4: a 2048x2048 field cut into 128x128 patches at stride 64 (961
    patches), 24 frames, four objects (one wideband and three narrowband
    channels at lambda/lambda_0 = 1.0, 0.95, 1.05, 1.1: pupil diameter and
    phases scaled by lambda_0/lambda), 150 modes (Noll 2..151), D/r0 = 15,
    and an object smoothness prior.
  * make_problem: the same recipe at any small size, for ragged test cases.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .fields import gaussian_noise, object_field
from .geometry import defocus_diversity, hann_window, pupil_mask, zernike_basis
from .turbulence import draw_kolmogorov

SEED_ROOT = 250510639


@dataclass
class Problem:
    """Inputs of one MOMFBD evaluation (C-order float arrays)."""

    N: int
    P: int
    C: int
    K: int
    J: int
    M: int
    channel_object: np.ndarray          # int32 [C]
    pupil: np.ndarray                   # float32 [C][N][N]
    basis: np.ndarray                   # float32 [C][M][N][N]  (rad)
    diversity: np.ndarray               # float32 [C][N][N]     (rad)
    alpha_true: np.ndarray              # float32 [P][J][M]
    window: np.ndarray                  # float32 [N][N]
    gamma: float
    weights: np.ndarray                 # float32 [C][J]
    objects: np.ndarray                 # float64 [P][K][N][N] true scenes
    noise: np.ndarray                   # float32 [P][C][J][N][N]
    d_over_r0: np.ndarray               # float64 [P]
    meta: dict = field(default_factory=dict)


def _streams(key):
    ss = np.random.SeedSequence([SEED_ROOT] + list(np.atleast_1d(key)))
    return [np.random.default_rng(s) for s in ss.spawn(4)]


def patch_grid(H: int, W: int, N: int, stride: int):
    """Top-left corners of the patch grid: y0 = i*stride, i = 0..(H-N)//stride."""
    ny = (H - N) // stride + 1
    nx = (W - N) // stride + 1
    ys = np.arange(ny) * stride
    xs = np.arange(nx) * stride
    return ys, xs


def make_problem(key, N=64, P=1, J=8, M=44, channels=((0, 0.0),),
                 d_over_r0=10.0, gamma=1e-3, border=6, noise_sigma=0.01,
                 diameter_frac=0.45, lam_ratios=None, objects=None) -> Problem:
    """Build a problem with independent periodic N x N scenes per patch.

    ``channels`` lists (object id, diversity in waves PV of defocus) per
    channel.  ``lam_ratios`` optionally gives lambda_0/lambda_c per channel:
    the basis and the diversity of that channel are scaled by it (wavefront
    equation of Sect. "Wavefronts") and its pupil diameter in pixels too.
    """
    rng_obj, rng_wf, rng_noise, _ = _streams(key)
    C = len(channels)
    chan_obj = np.array([c[0] for c in channels], dtype=np.int32)
    K = int(chan_obj.max()) + 1
    lam = np.ones(C) if lam_ratios is None else np.asarray(lam_ratios, float)
    # a channel at lambda_c = lambda_0 / lam[c] sees a pupil of diameter
    # d lam[c] pixels (sampling D pix / lambda) and phases scaled by lam[c]
    fracs = [diameter_frac * lam[c] for c in range(C)]
    A = np.stack([pupil_mask(N, fracs[c]) for c in range(C)])
    basis = np.stack([zernike_basis(N, M, fracs[c]) * lam[c] for c in range(C)])
    div = np.stack([defocus_diversity(N, channels[c][1], fracs[c]) * lam[c]
                    if channels[c][1] != 0.0 else np.zeros((N, N))
                    for c in range(C)])
    d_r0 = np.broadcast_to(np.asarray(d_over_r0, float), (P,)).copy()
    alpha = draw_kolmogorov(rng_wf, P * J, M, np.repeat(d_r0, J)).reshape(P, J, M)
    if objects is None:
        objects = np.stack([np.stack([object_field(rng_obj, N) for _ in range(K)])
                            for _ in range(P)])
    noise = gaussian_noise(rng_noise, (P, C, J, N, N), noise_sigma)
    return Problem(N=N, P=P, C=C, K=K, J=J, M=M, channel_object=chan_obj,
                   pupil=A.astype(np.float32),
                   basis=basis.astype(np.float32), diversity=div.astype(np.float32),
                   alpha_true=alpha.astype(np.float32),
                   window=hann_window(N, border).astype(np.float32), gamma=float(gamma),
                   weights=np.ones((C, J), np.float32), objects=objects,
                   noise=noise.astype(np.float32), d_over_r0=d_r0,
                   meta=dict(key=key, border=border, noise_sigma=noise_sigma,
                             diameter_frac=diameter_frac))


def config0() -> Problem:
    """One 64x64 patch, 1 object, 8 frames, 44 modes, D/r0 = 10."""
    return make_problem(0, N=64, P=1, J=8, M=44, channels=((0, 0.0),),
                        d_over_r0=10.0, gamma=1e-3, border=6)


def config1_geometry():
    """Sizes of the full-field workload: 1024^2 frames, 64^2 patches, stride 32."""
    H = W = 1024
    N, stride = 64, 32
    ys, xs = patch_grid(H, W, N, stride)
    return dict(H=H, W=W, N=N, stride=stride, ny=len(ys), nx=len(xs),
                P=len(ys) * len(xs), J=12, C=2, K=2, M=66, gamma=1e-3, border=6,
                channels=((0, 0.0), (1, 1.0)))


def config1_d_over_r0():
    g = config1_geometry()
    iy, ix = np.meshgrid(np.arange(g["ny"]), np.arange(g["nx"]), indexing="ij")
    return (5.0 + 15.0 * (ix + iy) / float((g["nx"] - 1) + (g["ny"] - 1))).ravel()


def config1_alpha() -> np.ndarray:
    """Modal coefficients [961][12][66] of the full-field workload (float32)."""
    g = config1_geometry()
    _, rng_wf, _, _ = _streams(1)
    d_r0 = config1_d_over_r0()
    a = draw_kolmogorov(rng_wf, g["P"] * g["J"], g["M"], np.repeat(d_r0, g["J"]))
    return a.reshape(g["P"], g["J"], g["M"]).astype(np.float32)


def config1_object(rng=None) -> np.ndarray:
    """The 1024x1024 k^-3 scene of the full-field workload (float64)."""
    g = config1_geometry()
    if rng is None:
        rng = _streams(1)[0]
    return object_field(rng, g["H"], g["W"])


def config1_problem(patches=None) -> Problem:
    """Full-field workload restricted to ``patches`` (indices; default all).

    Each patch's scene is its cut of the 1024^2 field; frames are formed
    patch by patch (isoplanatic inside a patch).  Noise is drawn for the
    selected patches only, from a stream keyed by the patch index, so any
    subset is reproducible on its own.
    """
    g = config1_geometry()
    N = g["N"]
    sel = np.arange(g["P"]) if patches is None else np.asarray(patches)
    scene = config1_object()
    ys, xs = patch_grid(g["H"], g["W"], N, g["stride"])
    objs = np.empty((len(sel), g["K"], N, N))
    for i, p in enumerate(sel):
        y0, x0 = ys[p // g["nx"]], xs[p % g["nx"]]
        objs[i, :] = scene[y0:y0 + N, x0:x0 + N]
    base = make_problem(1, N=N, P=1, J=g["J"], M=g["M"], channels=g["channels"],
                        gamma=g["gamma"], border=g["border"], objects=objs[:1])
    alpha = config1_alpha()[sel]
    noise = np.empty((len(sel), g["C"], g["J"], N, N), np.float32)
    for i, p in enumerate(sel):
        rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 1, 7, int(p)]))
        noise[i] = gaussian_noise(rng, (g["C"], g["J"], N, N), 0.01)
    base.P = len(sel)
    base.alpha_true = alpha
    base.objects = objs
    base.noise = noise
    base.d_over_r0 = config1_d_over_r0()[sel]
    base.meta.update(patches=sel, key=1)
    return base


def config4_geometry():
    """Sizes of the large multi-object workload: 2048^2, 128^2 patches, stride 64."""
    H = W = 2048
    N, stride = 128, 64
    ys, xs = patch_grid(H, W, N, stride)
    lam = (1.0, 1.0 / 0.95, 1.0 / 1.05, 1.0 / 1.1)       # lambda_0 / lambda_c
    return dict(H=H, W=W, N=N, stride=stride, ny=len(ys), nx=len(xs),
                P=len(ys) * len(xs), J=24, C=4, K=4, M=150, gamma=1e-3, smooth=1e-2,
                border=12, d_over_r0=15.0, lam_ratios=lam,
                channels=((0, 0.0), (1, 0.0), (2, 0.0), (3, 0.0)))


def config4_template() -> Problem:
    """Pupils, basis, window and channel map of the large workload (one patch)."""
    g = config4_geometry()
    N = g["N"]
    return make_problem(4, N=N, P=1, J=1, M=g["M"], channels=g["channels"], gamma=g["gamma"],
                        border=g["border"], lam_ratios=g["lam_ratios"],
                        objects=np.zeros((1, g["K"], N, N)))


def config4_alpha() -> np.ndarray:
    """Modal coefficients [961][24][150] of the large workload (float32)."""
    g = config4_geometry()
    _, rng_wf, _, _ = _streams(4)
    n = g["P"] * g["J"]
    a = draw_kolmogorov(rng_wf, n, g["M"], np.full(n, g["d_over_r0"]))
    return a.reshape(g["P"], g["J"], g["M"]).astype(np.float32)


def config4_objects() -> np.ndarray:
    """Four 2048x2048 k^-3 scenes, one per object (float32)."""
    g = config4_geometry()
    rng = _streams(4)[0]
    return np.stack([object_field(rng, g["H"], g["W"]).astype(np.float32)
                     for _ in range(g["K"])])


def config4_problem(patches) -> Problem:
    """Large multi-object workload restricted to ``patches`` (indices).

    Each patch's four scenes are its cuts of the four 2048^2 fields; its
    coefficients are its rows of ``config4_alpha``.  Noise is drawn per
    patch from a stream keyed by the patch index, so any subset is
    reproducible on its own.
    """
    g = config4_geometry()
    N = g["N"]
    sel = np.asarray(patches)
    scenes = config4_objects()
    ys, xs = patch_grid(g["H"], g["W"], N, g["stride"])
    objs = np.empty((len(sel), g["K"], N, N))
    for i, p in enumerate(sel):
        y0, x0 = ys[p // g["nx"]], xs[p % g["nx"]]
        objs[i] = scenes[:, y0:y0 + N, x0:x0 + N]
    base = config4_template()
    noise = np.empty((len(sel), g["C"], g["J"], N, N), np.float32)
    for i, p in enumerate(sel):
        rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 4, 7, int(p)]))
        noise[i] = gaussian_noise(rng, (g["C"], g["J"], N, N), 0.01)
    base.P, base.J = len(sel), g["J"]
    base.alpha_true = config4_alpha()[sel]
    base.objects = objs
    base.noise = noise
    base.weights = np.ones((g["C"], g["J"]), np.float32)
    base.d_over_r0 = np.full(len(sel), g["d_over_r0"])
    base.meta.update(patches=sel, key=4)
    return base
