"""Shared helpers for the tests: problem set-up and comparison metrics."""

from __future__ import annotations

import numpy as np

import oracle
import synth

# Tolerances of the GPU path against the FP64 oracle (FP32 arithmetic):
LOSS_RTOL = 1e-5        # relative, per patch
GRAD_RTOL = 1e-4        # ||g_gpu - g_ref||_2 / ||g_ref||_2, per patch
GRAD_ELEM = 1e-4        # max |g_gpu - g_ref| / max |g_ref|, per patch (every element)
OBJ_RMS = 1e-4          # rms of the restored object difference (frame units)


def simulate_D(pr: synth.Problem, threads: int = 8) -> np.ndarray:
    """Data spectra [P][C][J][N][N/2+1] complex64 of a problem, made by the oracle.

    Patches are simulated in chunks on a thread pool (numpy's matrix products
    release the GIL); the result does not depend on the chunking.
    """
    from concurrent.futures import ThreadPoolExecutor

    def one(sel):
        frames = oracle.simulate_frames(pr.objects[sel], pr.alpha_true[sel], pr.basis,
                                        pr.diversity, pr.pupil, pr.channel_object,
                                        pr.noise[sel])
        return oracle.patch_spectra(frames, pr.window).astype(np.complex64)

    chunks = [list(range(s, min(pr.P, s + 16))) for s in range(0, pr.P, 16)]
    if len(chunks) == 1:
        return one(chunks[0])
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(one, chunks))
    return np.concatenate(parts)


def fast_simulate_D(pr: synth.Problem) -> np.ndarray:
    """The same synthetic data as simulate_D, made with scipy.fft (input
    synthesis only; expected values always come from the oracle)."""
    import os

    from scipy import fft as sfft
    wk = min(16, os.cpu_count() or 1)
    N = pr.N
    A = pr.pupil.astype(np.float64)
    kap = 1.0 / (N * N * A.sum(axis=(1, 2)))
    Ok = sfft.fft2(pr.objects, workers=wk)
    out = np.empty((pr.P, pr.C, pr.J, N, N // 2 + 1), np.complex64)
    win = pr.window.astype(np.float64)
    for c in range(pr.C):
        phi = np.tensordot(pr.alpha_true.astype(np.float64), pr.basis[c].astype(np.float64),
                           axes=(2, 0)) + pr.diversity[c]
        p = sfft.ifft2(A[c] * np.exp(1j * phi), workers=wk) * (N * N)
        s = kap[c] * np.abs(p) ** 2
        img = sfft.ifft2(Ok[:, int(pr.channel_object[c])][:, None] * sfft.fft2(s, workers=wk),
                         workers=wk).real
        img += pr.noise[:, c]
        m = img.mean(axis=(-2, -1), keepdims=True)
        out[:, c] = sfft.rfft2(win * (img - m) + m, workers=wk)
    return out


def alpha_points(pr: synth.Problem, seed=0):
    """The three coefficient sets parity is checked at: 0, truth, perturbed truth."""
    rng = np.random.default_rng(seed)
    a0 = np.zeros_like(pr.alpha_true)
    a2 = (pr.alpha_true + 0.3 * rng.standard_normal(pr.alpha_true.shape)).astype(np.float32)
    return {"zero": a0, "true": pr.alpha_true.copy(), "perturbed": a2}


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def grad_errs(g_gpu, g_ref):
    return [rel_err(g_gpu[p], g_ref[p]) for p in range(g_ref.shape[0])]


def grad_elem_errs(g_gpu, g_ref):
    """Per patch: the largest element-wise gradient difference over the
    largest reference element, so that an error confined to one mode or one
    frame cannot hide in the norm."""
    out = []
    for p in range(g_ref.shape[0]):
        r = np.asarray(g_ref[p], np.float64)
        d = np.abs(np.asarray(g_gpu[p], np.float64) - r)
        out.append(float(d.max() / max(np.abs(r).max(), 1e-300)))
    return out


def assert_grad_close(g_gpu, g_ref, what=""):
    """Gradient parity per patch: the norm bound and the element bound."""
    gn = grad_errs(g_gpu, g_ref)
    ge = grad_elem_errs(g_gpu, g_ref)
    assert max(gn) < GRAD_RTOL, (what, "norm", max(gn))
    assert max(ge) < GRAD_ELEM, (what, "element", max(ge))
