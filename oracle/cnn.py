"""FP64 oracle of the warm-start network -- test infrastructure.

A plain NumPy forward and backward pass of the convolutional regressor that
maps a burst of frames to per-frame modal coefficients, written from the
definitions of convolution, ReLU and matrix products; no code shared with
the GPU library.  Activations are NHWC.

Network: conv 3x3 stride 2 padding 1 layers with ReLU, then dense layers
(ReLU on all but the last).  A conv layer's weight is [Co][3][3][Ci] and its
output is y[b, oy, ox, co] = bias[co] + sum_{ky,kx,ci} w[co, ky, kx, ci]
x[b, 2 oy + ky - 1, 2 ox + kx - 1, ci] (zero outside the image).  A dense
layer's weight is [out][in].  The first dense layer reads the last conv
output flattened in (y, x, c) order.

`bf16=True` rounds what the GPU stores in bfloat16 (inputs, weights,
activations, back-propagated activation gradients) to bfloat16 the way the
GPU does: the FP32 value rounded to nearest even.  Accumulations are FP64.

Loss (per frame, the coefficient of a frame cannot be recovered beyond two
symmetries of the problem): the tilt modes' mean over the burst is removed
from prediction and target (a common shift of all frames is not seen), and
the squared error is the smaller of those against the target and against
the target with its even modes negated (the PSF of phi(r) equals that of
-phi(-r); Sect. "Wavefronts" notes the sign ambiguity of even modes
without diversity).  Loss = mean over (burst, frame) of that minimum.  Mode
errors are weighted (by each mode's variance over the training set, so the
loss measures wavefront error rather than giving every mode equal say).
"""

from __future__ import annotations

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """FP32 rounding, then round to nearest even at 8 mantissa bits."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), f, out).astype(np.float64)


def conv_forward(x, w, b):
    """x [B][H][W][Ci], w [Co][3][3][Ci], b [Co] -> [B][H/2][W/2][Co]."""
    B, H, W, Ci = x.shape
    Ho, Wo = H // 2, W // 2
    xp = np.zeros((B, H + 2, W + 2, Ci))
    xp[:, 1:H + 1, 1:W + 1] = x
    y = np.broadcast_to(b, (B, Ho, Wo, w.shape[0])).copy()
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :]      # [B][Ho][Wo][Ci]
            y += patch @ w[:, ky, kx, :].T
    return y


def conv_backward(x, w, dy):
    """Gradients of conv_forward: (dx, dw, db)."""
    B, H, W, Ci = x.shape
    Ho, Wo = H // 2, W // 2
    xp = np.zeros((B, H + 2, W + 2, Ci))
    xp[:, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :]
            dw[:, ky, kx, :] = np.einsum("bhwo,bhwi->oi", dy, patch)
            dxp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2, :] += dy @ w[:, ky, kx, :]
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, 1:H + 1, 1:W + 1], dw, db


def even_mode_mask(M: int, first_noll: int = 2) -> np.ndarray:
    """True for modes of even radial order n (Noll j = first_noll..)."""
    out = np.zeros(M, bool)
    for i in range(M):
        j = first_noll + i
        n = 0
        while (n + 1) * (n + 2) // 2 < j:
            n += 1
        out[i] = n % 2 == 0
    return out


def burst_loss(pred, target, even, tilt=(0, 1), weight=None):
    """Loss and d loss / d pred; pred, target [B][J][M] (FP64); `weight` [M]
    weighs each mode's squared error (default 1)."""
    B, J, M = pred.shape
    t = np.asarray(tilt)
    p = pred.copy()
    q = target.astype(np.float64).copy()
    p[:, :, t] -= p[:, :, t].mean(axis=1, keepdims=True)
    q[:, :, t] -= q[:, :, t].mean(axis=1, keepdims=True)
    sign = np.where(even, -1.0, 1.0)
    wt = np.ones(M) if weight is None else np.asarray(weight, np.float64)
    e1 = np.sum(wt * (p - q) ** 2, axis=2)
    e2 = np.sum(wt * (p - q * sign) ** 2, axis=2)
    use2 = e2 < e1
    ref = np.where(use2[:, :, None], q * sign, q)
    loss = float(np.mean(np.minimum(e1, e2)))
    g = 2.0 * wt * (p - ref) / (B * J)
    # through the removal of the tilt mean
    g[:, :, t] -= g[:, :, t].mean(axis=1, keepdims=True)
    return loss, g, use2


def normalize_frames(frames):
    """[B][J][H][W] -> NHWC [B][H][W][J]: each frame divided by its mean,
    minus one, times ten."""
    m = frames.mean(axis=(2, 3), keepdims=True)
    x = 10.0 * (frames / m - 1.0)
    return np.transpose(x, (0, 2, 3, 1))


class Network:
    """Layer list [("conv", Ci, Co) ..., ("dense", n_in, n_out) ...]."""

    def __init__(self, layers):
        self.layers = layers

    def unpack(self, params):
        out, o = [], 0
        for kind, a, b in self.layers:
            nw = b * 9 * a if kind == "conv" else b * a
            w = params[o:o + nw].reshape((b, 3, 3, a) if kind == "conv" else (b, a))
            o += nw
            bias = params[o:o + b]
            o += b
            out.append((w, bias))
        return out

    def count(self):
        return sum((b * 9 * a if k == "conv" else b * a) + b for k, a, b in self.layers)

    def forward(self, x, params, bf16=False):
        rnd = bf16_round if bf16 else (lambda v: np.asarray(v, np.float64))
        # weights are stored in bfloat16, biases stay FP32
        wts = [(rnd(w), np.asarray(b, np.float64)) for w, b in self.unpack(params)]
        acts = [rnd(x)]
        h = acts[0]
        n = len(self.layers)
        for i, ((kind, _, _), (w, b)) in enumerate(zip(self.layers, wts)):
            if kind == "conv":
                z = conv_forward(h, w, b)
            else:
                z = h.reshape(h.shape[0], -1) @ w.T + b
            if i < n - 1:
                h = rnd(np.maximum(z, 0.0))
            else:
                h = z                                   # FP32 output of the last layer
            acts.append(h)
        return acts, wts

    def loss_grad(self, x, params, target, even, bf16=False, weight=None):
        """Loss and gradient with respect to the (FP32 master) parameters."""
        rnd = bf16_round if bf16 else (lambda v: np.asarray(v, np.float64))
        acts, wts = self.forward(x, params, bf16)
        B, J, M = target.shape
        pred = acts[-1].reshape(B, J, M)
        loss, g, _ = burst_loss(pred, target, even, weight=weight)
        grads = []
        dz = rnd(g.reshape(B, -1))
        n = len(self.layers)
        for i in range(n - 1, -1, -1):
            kind = self.layers[i][0]
            w, _ = wts[i]
            h_in = acts[i]
            if kind == "dense":
                hin = h_in.reshape(B, -1)
                dw = dz.T @ hin
                db = dz.sum(axis=0)
                dh = dz @ w
                dh = dh.reshape(h_in.shape)
            else:
                dh, dw, db = conv_backward(h_in, w, dz)
            grads.append((dw, db))
            if i > 0:
                dz = rnd(dh * (h_in > 0))
        grads.reverse()
        flat = np.concatenate([np.concatenate([dw.ravel(), db.ravel()]) for dw, db in grads])
        return loss, flat, pred
