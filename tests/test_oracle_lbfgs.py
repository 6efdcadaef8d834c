"""Pins of the reference L-BFGS solver (Nocedal & Wright Alg. 7.4 + 3.5/3.6)."""

import numpy as np

import oracle
import synth
from oracle.lbfgs import cubic_min, wolfe_search


def test_cubic_interpolation_is_exact_for_cubics():
    f = lambda t: (t - 0.3) ** 2 * (t + 2.0)            # local min at t = 0.3
    g = lambda t: 2 * (t - 0.3) * (t + 2.0) + (t - 0.3) ** 2
    t = cubic_min(0.0, f(0.0), g(0.0), 1.0, f(1.0), g(1.0))
    assert abs(t - 0.3) < 1e-12


def test_quadratic_converges_to_closed_form():
    rng = np.random.default_rng(0)
    Q = rng.standard_normal((12, 12))
    A = Q @ Q.T + 12 * np.eye(12)
    b = rng.standard_normal(12)
    fg = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    x, f, _ = oracle.lbfgs_minimize(fg, np.zeros(12), max_iter=200)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), atol=1e-8)


def test_rosenbrock():
    def fg(x):
        f = 100 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
        g = np.array([-400 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]), 200 * (x[1] - x[0] ** 2)])
        return f, g
    x, f, _ = oracle.lbfgs_minimize(fg, np.array([-1.2, 1.0]), max_iter=500)
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-6)


def test_strong_wolfe_conditions_hold():
    fg = lambda x: (np.sum(np.cosh(x)), np.sinh(x))
    x = np.array([1.0, -2.0, 0.5])
    f0, g0 = fg(x)
    d = -g0
    t, f, g, n, ok = wolfe_search(fg, x, f0, g0, d, 1.0)
    assert ok
    assert f <= f0 + 1e-4 * t * (g0 @ d)
    assert abs(g @ d) <= 0.9 * abs(g0 @ d)


def test_momfbd_config0_descends_below_true_coefficients():
    pr = synth.config0()
    frames = oracle.simulate_frames(pr.objects, pr.alpha_true, pr.basis, pr.diversity,
                                    pr.pupil, pr.channel_object, pr.noise)
    D = oracle.patch_spectra(frames, pr.window).astype(np.complex64)
    shape = pr.alpha_true[0].shape

    def fg(x):
        r = oracle.evaluate_patch(x.reshape(shape), D[0], pr.basis, pr.diversity, pr.pupil,
                                  pr.channel_object, pr.gamma)
        return r["loss"], r["grad"].ravel()

    l_true = fg(pr.alpha_true[0].astype(np.float64).ravel())[0]
    x, f, hist = oracle.lbfgs_minimize(fg, np.zeros(np.prod(shape)), max_iter=150)
    assert all(b <= a for a, b in zip(hist, hist[1:]))
    assert f < l_true, (f, l_true)
