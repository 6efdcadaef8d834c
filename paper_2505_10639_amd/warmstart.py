"""Learned warm start for MOMFBD: libmomfbd's convolutional regressor,
trained on bursts made by the library's own forward model
(momfbd_synthesize), and used as the start point of the per-patch L-BFGS.

All arithmetic runs in libmomfbd's kernels, random normals included
(momfbd_random_normal); this module allocates tensors, draws the per-burst
parameters (turbulence strength, noise level, scene crop) on the host from
a seeded generator, and sequences calls.
"""

from __future__ import annotations

import time

import numpy as np
import torch

from . import _lib
from .plan import Plan, Solver


# generator streams of the library's normal draws
STREAM_INIT, STREAM_NOISE = 0x1417, 0x2050


class WarmStartNet:
    """The network with its FP32 parameters, Adam moments and workspace.
    N: side of the input frames (64, 96 or 128); J frames; M modes (the
    lowest M of the solve)."""

    def __init__(self, J, M, mode_scale, batch_max=256, device="cuda:0", N=64):
        self.device = torch.device(device)
        self.N, self.J, self.M, self.batch_max = int(N), int(J), int(M), int(batch_max)
        self.mode_scale = np.asarray(mode_scale, np.float32)
        with torch.cuda.device(self.device):
            self.handle = _lib.momfbd_cnn_create(self.N, self.J, self.M, self.batch_max,
                                                 self.mode_scale)
            n_params, ws_bytes = _lib.momfbd_cnn_sizes(self.handle)
            self.n_params = n_params
            self.params = torch.zeros(n_params, dtype=torch.float32, device=self.device)
            self.m1 = torch.zeros_like(self.params)
            self.m2 = torch.zeros_like(self.params)
            self.grad = torch.zeros_like(self.params)
            self.ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=self.device)
            self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.steps = 0

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _lib.momfbd_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, seed: int):
        normals = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _lib.momfbd_random_normal(int(seed), STREAM_INIT, 0, normals)
        _lib.momfbd_cnn_init(self.handle, normals, self.params, self.ws)
        self.m1.zero_()
        self.m2.zero_()
        self.steps = 0

    def load(self, params):
        self.params.copy_(torch.as_tensor(params, dtype=torch.float32, device=self.device))
        _lib.momfbd_cnn_load(self.handle, self.params, self.ws)

    def predict(self, D):
        """alpha [B][J][M] from data spectra D [B][C][J][N][N/2+1] (the
        network reads channel 0)."""
        B, C = D.shape[0], D.shape[1]
        out = torch.empty((B, self.J, self.M), dtype=torch.float32, device=self.device)
        for b0 in range(0, B, self.batch_max):
            b1 = min(B, b0 + self.batch_max)
            _lib.momfbd_cnn_forward(self.handle, self.params, D[b0:b1], b1 - b0, C, out[b0:b1],
                                    self.ws)
        return out

    def input(self, D):
        """The network's input x [B][N][N][J] for data spectra D (bfloat16
        values as floats; momfbd_cnn_input)."""
        B, C = D.shape[0], D.shape[1]
        x = torch.empty((B, self.N, self.N, self.J), dtype=torch.float32, device=self.device)
        for b0 in range(0, B, self.batch_max):
            b1 = min(B, b0 + self.batch_max)
            _lib.momfbd_cnn_input(self.handle, D[b0:b1], b1 - b0, C, x[b0:b1], self.ws)
        return x

    def loss_grad(self, D, target):
        _lib.momfbd_cnn_loss_grad(self.handle, self.params, D, D.shape[1], target, D.shape[0],
                                  self.loss, self.grad, self.ws)
        return self.loss, self.grad

    def train_step(self, D, target, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.loss_grad(D, target)
        self.steps += 1
        _lib.momfbd_cnn_adam(self.handle, self.params, self.grad, self.m1, self.m2, self.steps, lr,
                             beta1, beta2, eps, self.ws)
        return self.loss


class BurstSource:
    """Bursts of the single-object N x N forward model (one channel: the
    given pupil and basis): object crops of large k^-3 scenes (their spectra
    precomputed on the GPU), Kolmogorov wavefronts with D/r0 uniform in
    [r_lo, r_hi], white noise with SNR uniform in [snr_lo, snr_hi] (relative
    to the unit scene mean) drawn by the library's generator."""

    def __init__(self, pupil, basis, window, J, batch, scenes, crop_stride=16, seed=0,
                 r0_range=(4.0, 20.0), snr_range=(50.0, 200.0), device="cuda:0"):
        import synth
        self.device = torch.device(device)
        self.N = int(np.asarray(pupil).shape[-1])
        N, H2 = self.N, self.N // 2 + 1
        self.J, self.batch = int(J), int(batch)
        self.M = int(np.asarray(basis).shape[1])
        self.r0_range, self.snr_range = r0_range, snr_range
        self.rng = np.random.default_rng(seed)
        self.seed = int(seed)
        self.counter = 0
        self.plan = Plan(N, self.batch, self.J, [0], pupil, basis, None, self.device)
        self.window = torch.as_tensor(np.asarray(window, np.float32), device=self.device)
        self.noise = torch.empty((self.batch, 1, self.J, N, N), dtype=torch.float32,
                                 device=self.device)
        ones = torch.ones((N, N), dtype=torch.float32, device=self.device)
        banks = []
        for sc in scenes:
            H, W = sc.shape
            ny, nx = (H - N) // crop_stride + 1, (W - N) // crop_stride + 1
            aux = Plan(N, ny * nx, 1, [0], pupil, np.asarray(basis)[:, :1], None, self.device)
            t = torch.as_tensor(np.asarray(sc, np.float32), device=self.device)
            banks.append(aux.prepare_data(t.reshape(1, 1, H, W).contiguous(), crop_stride, ones)
                         .reshape(ny * nx, 1, N, H2))
            aux.close()
        self.bank = torch.cat(banks)
        self._draw = synth.draw_kolmogorov

    def next(self):
        """(D [B][1][J][N][N/2+1], alpha [B][J][M]) of a fresh batch."""
        B, J, M = self.batch, self.J, self.M
        r0 = self.rng.uniform(*self.r0_range, size=B)
        alpha = self._draw(self.rng, B * J, M, np.repeat(r0, J)).reshape(B, J, M)
        alpha = torch.as_tensor(alpha.astype(np.float32), device=self.device)
        idx = torch.as_tensor(self.rng.integers(0, self.bank.shape[0], size=B), device=self.device)
        O = self.bank[idx].contiguous()
        snr = self.rng.uniform(*self.snr_range, size=B)
        sigma = torch.as_tensor((1.0 / snr).astype(np.float32), device=self.device)
        _lib.momfbd_random_normal(self.seed, STREAM_NOISE, self.counter, self.noise)
        self.counter += self.noise.numel() // 4
        _, D = self.plan.synthesize(alpha, O, self.noise, sigma, self.window)
        return D, alpha

    def close(self):
        self.plan.close()


def mode_scale(M, r0_range=(4.0, 20.0), ao_modes=9, ao_factor=0.3):
    """Standard deviation of each mode over the training distribution:
    sqrt(Noll variance) * sqrt(E[(D/r0)^(5/3)]) (times ao_factor for the
    first ao_modes modes)."""
    import synth
    var = np.diag(synth.noll_covariance(M))
    lo, hi = r0_range
    e = (hi ** (8 / 3) - lo ** (8 / 3)) / ((8 / 3) * (hi - lo))
    s = np.sqrt(var * e)
    s[:ao_modes] *= ao_factor
    return s.astype(np.float32)


def solve_rounds_until(plan, alpha0, D, gamma, target_loss=None, max_rounds=6000, chunk=8,
                       stall=5, rtol=1e-10):
    """Per-patch L-BFGS from alpha0 in solver rounds (momfbd_lbfgs_rounds:
    each round gives every running patch one line-search trial, with no host
    synchronisation), `chunk` rounds between reads of the summed accepted
    loss.  Stops when that sum is <= target_loss, or (no target) when it
    changes by less than rtol over `stall` chunks, or after max_rounds.
    Patches do not wait for one another's line searches, so a round costs
    one evaluation of the running patches.  Returns (history of sums, one
    per chunk, seconds, accepted alpha, rounds run)."""
    alpha = alpha0.clone().contiguous()
    accepted = torch.empty_like(alpha)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol = Solver(plan, alpha, D, gamma)
    hist = [float(sol.loss.sum())]
    rounds = 0
    while rounds < max_rounds:
        loss, _ = sol.rounds(chunk)
        rounds += chunk
        hist.append(float(loss.sum()))
        if target_loss is not None and hist[-1] <= target_loss:
            break
        if target_loss is None and len(hist) > stall and \
                abs(hist[-1 - stall] - hist[-1]) <= rtol * abs(hist[-1]):
            break
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sol.rounds(0, accepted)
    return hist, elapsed, accepted, rounds


def solve_until(plan, alpha0, D, gamma, target_loss=None, max_iter=300, stall=20, rtol=1e-10):
    """Per-patch L-BFGS from alpha0.  Stops when sum_p L_p <= target_loss, or
    (no target) when the summed loss changes by less than rtol over `stall`
    iterations, or after max_iter.  Returns (history of sums, seconds, alpha)."""
    alpha = alpha0.clone().contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol = Solver(plan, alpha, D, gamma)
    hist = [float(sol.loss.sum())]
    for _ in range(max_iter):
        loss, _ = sol.step()
        hist.append(float(loss.sum()))
        if target_loss is not None and hist[-1] <= target_loss:
            break
        if target_loss is None and len(hist) > stall and \
                abs(hist[-1 - stall] - hist[-1]) <= rtol * abs(hist[-1]):
            break
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0, alpha
