"""Convenience wrapper: a plan with its workspace, checked tensor arguments.

Every computation runs in libmomfbd's kernels; this module only checks
shapes, dtypes and devices, allocates outputs with torch and passes
pointers.
"""

from __future__ import annotations

import numpy as np
import torch

from . import _lib


def _need(t, shape, dtype, name, device):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype} != {dtype}")
    if t.device != device:
        raise ValueError(f"{name}: device {t.device} != {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Plan:
    """A libmomfbd plan on one GPU plus a workspace tensor.

    pupil [C][N][N], basis [C][M][N][N] (rad), diversity [C][N][N] (rad) or
    None are host (numpy) arrays; channel_object lists the object of each
    channel.
    """

    def __init__(self, N, P, J, channel_object, pupil, basis, diversity=None, device="cuda:0"):
        self.device = torch.device(device)
        channel_object = [int(v) for v in channel_object]
        self.N, self.P, self.J = int(N), int(P), int(J)
        self.C = len(channel_object)
        self.K = max(channel_object) + 1
        self.M = int(np.asarray(basis).shape[1])
        with torch.cuda.device(self.device):
            self.handle = _lib.momfbd_plan_create(self.N, self.P, self.C, self.K, self.J, self.M,
                                                  channel_object, pupil, basis, diversity)
            nbytes = _lib.momfbd_workspace_size(self.handle)
            self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)

    def object_filtered(self, alpha, D, filters, gamma=1e-3, weights=None, want_H=False):
        """Restored objects [P][K][N][N] after one Fourier filter per object
        (`filters`: K specs from filter_spec); with want_H also the filters
        [P][K][N][N/2+1]."""
        self._alpha(alpha)
        self._D(D)
        g_arr, g_sc = self._gamma(gamma)
        self._weights(weights)
        if len(filters) != self.K:
            raise ValueError(f"{len(filters)} filters for {self.K} objects")
        obj = torch.empty((self.P, self.K, self.N, self.N), dtype=torch.float32,
                          device=self.device)
        H = torch.empty((self.P, self.K) + self.half, dtype=torch.float32,
                        device=self.device) if want_H else None
        _lib.momfbd_object_filtered(self.handle, alpha, D, g_arr, g_sc, weights, list(filters),
                                    obj, H, self.ws)
        return (obj, H) if want_H else obj

    def mosaic(self, obj, ny, nx, stride, border):
        """Weighted mosaic [K][(ny-1)*stride+N][(nx-1)*stride+N] of restored
        patches obj [P][K][N][N]."""
        _need(obj, (self.P, self.K, self.N, self.N), torch.float32, "obj", self.device)
        out = torch.empty((self.K, (ny - 1) * stride + self.N, (nx - 1) * stride + self.N),
                          dtype=torch.float32, device=self.device)
        _lib.momfbd_mosaic(self.handle, obj, ny, nx, stride, border, out)
        return out

    def synthesize(self, alpha, O, noise, sigma, apod):
        """Bursts through the forward model: returns (frames [C][J][P*N][N],
        D [P][C][J][N][N/2+1])."""
        self._alpha(alpha)
        _need(O, (self.P, self.K) + self.half, torch.complex64, "O", self.device)
        _need(noise, (self.P, self.C, self.J, self.N, self.N), torch.float32, "noise", self.device)
        _need(sigma, (self.P,), torch.float32, "sigma", self.device)
        _need(apod, (self.N, self.N), torch.float32, "apod", self.device)
        frames = torch.empty((self.C, self.J, self.P * self.N, self.N), dtype=torch.float32,
                             device=self.device)
        D = torch.empty((self.P, self.C, self.J) + self.half, dtype=torch.complex64,
                        device=self.device)
        _lib.momfbd_synthesize(self.handle, alpha, O, noise, sigma, apod, frames, D, self.ws)
        return frames, D

    def tuning(self):
        return _lib.momfbd_plan_get_tuning(self.handle)

    def set_tuning(self, xcd_forward, xcd_adjoint, object_pairs_per_thread, grad_waves,
                   grad_splits=0, grad_row_tiles=0, phase_col_tiles=0, phase_waves=0,
                   object_fused=0):
        """Launch schedules (see momfbd_tuning); grad_splits 0 is automatic,
        grad_row_tiles 0 the default for the waves, phase_col_tiles and
        phase_waves 0 the widest phase block that fits, object_fused 1 the
        forward and object pass in one launch where the plan allows it."""
        _lib.momfbd_plan_set_tuning(self.handle, xcd_forward, xcd_adjoint,
                                    object_pairs_per_thread, grad_waves, grad_splits,
                                    grad_row_tiles, phase_col_tiles, phase_waves, object_fused)

    def autotune(self, alpha, D, gamma=1e-3, weights=None, reps=5):
        """Time the launch schedules on this data and keep the fastest."""
        self._alpha(alpha)
        self._D(D)
        g_arr, g_sc = self._gamma(gamma)
        self._weights(weights)
        loss = torch.empty(self.P, dtype=torch.float64, device=self.device)
        grad = torch.empty((self.P, self.J, self.M), dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            return _lib.momfbd_plan_autotune(self.handle, alpha, D, g_arr, g_sc, weights, reps,
                                             loss, grad, self.ws)

    def smoothness_gamma(self, gamma0, lam):
        """Per-frequency gamma [K][N][N/2+1] of the object smoothness prior
        for objects with constants gamma0[K] and lambda[K]."""
        g0 = np.broadcast_to(np.asarray(gamma0, np.float32), (self.K,))
        lm = np.broadcast_to(np.asarray(lam, np.float32), (self.K,))
        out = torch.empty((self.K,) + self.half, dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            _lib.momfbd_smoothness_gamma(self.handle, g0, lm, out)
        return out

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _lib.momfbd_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes
    @property
    def half(self):
        return (self.N, self.N // 2 + 1)

    def _alpha(self, alpha):
        return _need(alpha, (self.P, self.J, self.M), torch.float32, "alpha", self.device)

    def _D(self, D):
        return _need(D, (self.P, self.C, self.J) + self.half, torch.complex64, "D", self.device)

    def _gamma(self, gamma):
        if gamma is None or isinstance(gamma, (int, float)):
            return None, float(0.0 if gamma is None else gamma)
        return _need(gamma, (self.K,) + self.half, torch.float32, "gamma", self.device), 0.0

    def _weights(self, w):
        return _need(w, (self.C, self.J), torch.float32, "weights", self.device)

    def prepare_data(self, frames, stride, apod, D=None):
        C, J, H, W = frames.shape
        _need(frames, (self.C, self.J, H, W), torch.float32, "frames", self.device)
        _need(apod, (self.N, self.N), torch.float32, "apod", self.device)
        if D is None:
            D = torch.empty((self.P, self.C, self.J) + self.half, dtype=torch.complex64,
                            device=self.device)
        self._D(D)
        _lib.momfbd_prepare_data(self.handle, frames, H, W, stride, apod, D, self.ws)
        return D

    def forward(self, alpha, want_psf=True, want_otf=True):
        self._alpha(alpha)
        shp = (self.P, self.C, self.J)
        psf = torch.empty(shp + (self.N, self.N), dtype=torch.float32,
                          device=self.device) if want_psf else None
        otf = torch.empty(shp + self.half, dtype=torch.complex64,
                          device=self.device) if want_otf else None
        _lib.momfbd_forward(self.handle, alpha, psf, otf, self.ws)
        return psf, otf

    def loss_grad(self, alpha, D, gamma=1e-3, weights=None, want_grad=True, loss=None, grad=None):
        self._alpha(alpha)
        self._D(D)
        g_arr, g_sc = self._gamma(gamma)
        self._weights(weights)
        if loss is None:
            loss = torch.empty(self.P, dtype=torch.float64, device=self.device)
        if want_grad and grad is None:
            grad = torch.empty((self.P, self.J, self.M), dtype=torch.float32, device=self.device)
        _lib.momfbd_loss_grad(self.handle, alpha, D, g_arr, g_sc, weights, loss,
                              grad if want_grad else None, self.ws)
        return loss, (grad if want_grad else None)

    def object_estimate(self, alpha, D, gamma=1e-3, weights=None):
        self._alpha(alpha)
        self._D(D)
        g_arr, g_sc = self._gamma(gamma)
        self._weights(weights)
        obj = torch.empty((self.P, self.K, self.N, self.N), dtype=torch.float32,
                          device=self.device)
        _lib.momfbd_object_estimate(self.handle, alpha, D, g_arr, g_sc, weights, obj, self.ws)
        return obj


class Solver:
    """Per-patch L-BFGS on a plan (momfbd_lbfgs_init / momfbd_lbfgs_step).

    alpha (device float32 [P][J][M]) is updated in place by step().
    """

    def __init__(self, plan: Plan, alpha, D, gamma=1e-3, weights=None, m=10, max_evals=20,
                 c1=1e-4, c2=0.9, ftol=0.0):
        self.plan = plan
        self.alpha = plan._alpha(alpha)
        self.D = plan._D(D)
        self.gamma_arr, self.gamma_sc = plan._gamma(gamma)
        self.weights = plan._weights(weights)
        self.params = _lib.lbfgs_params(m, max_evals, c1, c2, ftol)
        nbytes = _lib.momfbd_lbfgs_state_size(plan.handle, self.params)
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=plan.device)
        self.loss = torch.empty(plan.P, dtype=torch.float64, device=plan.device)
        self.status = torch.zeros(plan.P, dtype=torch.int32, device=plan.device)
        _lib.momfbd_lbfgs_init(plan.handle, self.params, self.state, self.alpha, self.D,
                               self.gamma_arr, self.gamma_sc, self.weights, self.loss, plan.ws)

    def rounds(self, n, alpha_accepted=None):
        """n solver rounds (one line-search trial per running patch each)
        with no host synchronisation; capturable in a HIP graph."""
        _lib.momfbd_lbfgs_rounds(self.plan.handle, self.params, self.state, self.alpha, self.D,
                                 self.gamma_arr, self.gamma_sc, self.weights, n, self.loss,
                                 self.status, alpha_accepted, self.plan.ws)
        return self.loss, self.status

    def step(self):
        _lib.momfbd_lbfgs_step(self.plan.handle, self.params, self.state, self.alpha, self.D,
                               self.gamma_arr, self.gamma_sc, self.weights, self.loss,
                               self.status, self.plan.ws)
        return self.loss, self.status
