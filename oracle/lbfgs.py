"""Reference L-BFGS with a strong-Wolfe line search -- test infrastructure.

The paper minimises the summed patch loss with Adam (Sect. "Optimization and
paralellization"); the patches are independent because no coefficient is
shared between them.  The solver here is the quasi-Newton alternative: the
two-loop recursion of limited-memory BFGS and a bracketing/zoom line search
enforcing the strong Wolfe conditions (Nocedal & Wright, Numerical
Optimization, 2nd ed., Algorithms 7.4, 3.5 and 3.6), run per patch.
All scalars are float64.

Trial steps inside the zoom are the minimiser of the cubic through the two
bracket ends (values and slopes), clamped to the central 80% of the bracket;
bisection when the cubic has no real minimiser there.  The first trial step
of the first iteration is min(1, 1/||g||_inf); later iterations try 1.
"""

from __future__ import annotations

import math

import numpy as np


def cubic_min(a, fa, ga, b, fb, gb):
    """Minimiser of the cubic interpolating (a, fa, ga), (b, fb, gb), clamped
    to [lo + 0.1 w, hi - 0.1 w] of the bracket; midpoint if undefined."""
    lo, hi = (a, b) if a < b else (b, a)
    w = hi - lo
    d1 = ga + gb - 3.0 * (fa - fb) / (a - b)
    disc = d1 * d1 - ga * gb
    if disc >= 0.0 and w > 0.0:
        d2 = math.copysign(math.sqrt(disc), b - a)
        den = gb - ga + 2.0 * d2
        if den != 0.0:
            t = b - (b - a) * (gb + d2 - d1) / den
            if math.isfinite(t):
                return min(max(t, lo + 0.1 * w), hi - 0.1 * w)
    return 0.5 * (lo + hi)


def two_loop(g, S, Y):
    """Direction d = -H g from the stored pairs (oldest first)."""
    q = np.array(g, dtype=np.float64)
    k = len(S)
    alpha = np.zeros(k)
    rho = [1.0 / float(np.dot(Y[i], S[i])) for i in range(k)]
    for i in range(k - 1, -1, -1):
        alpha[i] = rho[i] * float(np.dot(S[i], q))
        q -= alpha[i] * Y[i]
    if k:
        q *= float(np.dot(S[-1], Y[-1])) / float(np.dot(Y[-1], Y[-1]))
    for i in range(k):
        beta = rho[i] * float(np.dot(Y[i], q))
        q += (alpha[i] - beta) * S[i]
    return -q


def wolfe_search(fg, x, f0, g0, d, t0, c1=1e-4, c2=0.9, max_eval=20):
    """Strong-Wolfe line search along d; returns (t, f, g, n_eval, ok)."""
    dphi0 = float(np.dot(g0, d))
    t_prev, f_prev, dphi_prev = 0.0, f0, dphi0
    t = t0
    n = 0

    def zoom(lo, flo, glo, hi, fhi, ghi, n):
        while n < max_eval:
            tj = cubic_min(lo, flo, glo, hi, fhi, ghi)
            fj, gj = fg(x + tj * d)
            n += 1
            dj = float(np.dot(gj, d))
            if fj > f0 + c1 * tj * dphi0 or fj >= flo:
                hi, fhi, ghi = tj, fj, dj
            else:
                if abs(dj) <= -c2 * dphi0:
                    return tj, fj, gj, n, True
                if dj * (hi - lo) >= 0.0:
                    hi, fhi, ghi = lo, flo, glo
                lo, flo, glo = tj, fj, dj
        return lo, None, None, n, False

    first = True
    while n < max_eval:
        ft, gt = fg(x + t * d)
        n += 1
        dt = float(np.dot(gt, d))
        if ft > f0 + c1 * t * dphi0 or (not first and ft >= f_prev):
            return zoom(t_prev, f_prev, dphi_prev, t, ft, dt, n)
        if abs(dt) <= -c2 * dphi0:
            return t, ft, gt, n, True
        if dt >= 0.0:
            return zoom(t, ft, dt, t_prev, f_prev, dphi_prev, n)
        t_prev, f_prev, dphi_prev = t, ft, dt
        t = 2.0 * t
        first = False
    return t_prev, None, None, n, False


def lbfgs_minimize(fg, x0, m=10, c1=1e-4, c2=0.9, max_iter=100, max_eval=20,
                   ftol=0.0, callback=None):
    """Minimise f with L-BFGS; fg(x) -> (f, g).  Returns (x, f, history)."""
    x = np.array(x0, dtype=np.float64)
    f, g = fg(x)
    S, Y = [], []
    hist = [f]
    for it in range(max_iter):
        d = two_loop(g, S, Y)
        if float(np.dot(g, d)) >= 0.0:       # not a descent direction: restart
            S, Y = [], []
            d = -g
        gmax = float(np.max(np.abs(g)))
        if gmax == 0.0:
            break
        t0 = min(1.0, 1.0 / gmax) if not S else 1.0
        t, fn, gn, _, ok = wolfe_search(fg, x, f, g, d, t0, c1, c2, max_eval)
        if fn is None:
            break
        s = t * d
        y = gn - g
        if float(np.dot(s, y)) > 1e-12 * float(np.dot(y, y)):
            S.append(s)
            Y.append(y)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        x = x + s
        df = f - fn
        f, g = fn, gn
        hist.append(f)
        if callback is not None:
            callback(it, x, f)
        if ftol > 0.0 and df <= ftol * max(abs(f), 1e-300):
            break
    return x, f, hist
