"""Pins of the warm-start network oracle: convolution against scipy, the
backward pass against central differences, the loss's invariances, and the
bfloat16 rounding rule."""

import numpy as np
from scipy import signal

from oracle import cnn


def test_bf16_round_to_nearest_even():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 3.0e38, 1e-40])
    r = cnn.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # tie -> even mantissa
    assert r[2] == 1 + 2 ** -6               # tie -> even mantissa (upwards)
    assert r[3] == 1 + 2 ** -7               # representable
    assert r[4] == -2.5
    assert np.isfinite(r[5]) and abs(r[5] / 3.0e38 - 1) < 2 ** -8
    assert r[6] == 2.0 ** -133                # subnormal: nearest multiple of 2^-133


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((10, 12))
    w = rng.standard_normal((3, 3))
    y = cnn.conv_forward(x[None, :, :, None], w[None, :, :, None], np.array([0.5]))[0, :, :, 0]
    ref = signal.correlate2d(x, w, mode="same")[::2, ::2] + 0.5
    np.testing.assert_allclose(y, ref, atol=1e-13)
    # channels add up
    x3 = rng.standard_normal((1, 8, 8, 3))
    w3 = rng.standard_normal((2, 3, 3, 3))
    y3 = cnn.conv_forward(x3, w3, np.zeros(2))
    for o in range(2):
        ref = sum(signal.correlate2d(x3[0, :, :, c], w3[o, :, :, c], mode="same")[::2, ::2]
                  for c in range(3))
        np.testing.assert_allclose(y3[0, :, :, o], ref, atol=1e-12)


def _tiny():
    net = cnn.Network([("conv", 3, 4), ("conv", 4, 5), ("dense", 20, 6), ("dense", 6, 6)])
    rng = np.random.default_rng(1)
    params = 0.4 * rng.standard_normal(net.count())
    x = rng.standard_normal((2, 8, 8, 3))
    target = rng.standard_normal((2, 2, 3))
    return net, params, x, target


def test_backward_matches_central_differences():
    net, params, x, target = _tiny()
    even = cnn.even_mode_mask(3)                  # Noll 2, 3, 4: tilt, tilt, defocus
    assert list(even) == [False, False, True]
    loss, grad, _ = net.loss_grad(x, params, target, even)
    h = 1e-6
    fd = np.empty_like(params)
    for i in range(len(params)):
        e = np.zeros_like(params)
        e[i] = h
        fd[i] = (net.loss_grad(x, params + e, target, even)[0]
                 - net.loss_grad(x, params - e, target, even)[0]) / (2 * h)
    np.testing.assert_allclose(grad, fd, rtol=1e-6, atol=1e-8)


def test_loss_invariances():
    rng = np.random.default_rng(2)
    B, J, M = 3, 4, 10
    even = cnn.even_mode_mask(M)
    p = rng.standard_normal((B, J, M))
    t = rng.standard_normal((B, J, M))
    l0 = cnn.burst_loss(p, t, even)[0]
    # flipping the even modes of any one frame of the target changes nothing
    t2 = t.copy()
    t2[1, 2, even] *= -1
    assert abs(cnn.burst_loss(p, t2, even)[0] - l0) < 1e-12
    # a tilt common to all frames of a burst changes nothing
    p2 = p.copy()
    p2[0, :, 0] += 0.7
    p2[2, :, 1] -= 1.3
    assert abs(cnn.burst_loss(p2, t, even)[0] - l0) < 1e-12
    # the loss is zero at the target
    assert cnn.burst_loss(t, t, even)[0] == 0.0


def test_weighted_loss_gradient_central_differences():
    rng = np.random.default_rng(7)
    B, J, M = 2, 3, 6
    even = cnn.even_mode_mask(M)
    wt = rng.uniform(0.2, 3.0, M)
    p = rng.standard_normal((B, J, M))
    t = rng.standard_normal((B, J, M))
    _, g, _ = cnn.burst_loss(p, t, even, weight=wt)
    h = 1e-7
    fd = np.empty_like(p)
    for i in np.ndindex(p.shape):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (cnn.burst_loss(p + e, t, even, weight=wt)[0]
                 - cnn.burst_loss(p - e, t, even, weight=wt)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)
    # unit weights reproduce the plain loss
    assert cnn.burst_loss(p, t, even, weight=np.ones(M))[0] == cnn.burst_loss(p, t, even)[0]


def test_bf16_network_close_to_fp64():
    net, params, x, target = _tiny()
    even = cnn.even_mode_mask(3)
    l64, g64, _ = net.loss_grad(x, params, target, even)
    l16, g16, _ = net.loss_grad(x, params, target, even, bf16=True)
    assert abs(l16 - l64) < 2e-2 * abs(l64)
    assert np.linalg.norm(g16 - g64) < 3e-2 * np.linalg.norm(g64)
