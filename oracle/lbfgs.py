"""L-BFGS with a strong-Wolfe line search, FP64 (oracle; test infrastructure only).

The paper solves eq. Thm5 with L-BFGS keeping 10 pairs in memory (Sec. 5.1,
Table 1) and defers the algorithm to Nocedal & Wright, which it cites.  This
module follows that textbook description:

* direction by the two-loop recursion with initial matrix gamma*I,
  gamma = s^T y / y^T y of the newest pair;
* step length by the strong-Wolfe bracketing/zoom search with cubic
  interpolation (c1 = 1e-4, c2 = 0.9), first trial alpha = 1 except
  min(1, 1/||g||_1) on the first iteration;
* a pair is stored only if s^T y > 1e-10 ||s|| ||y||;
* stop on ||g||_inf <= gtol * max(1, |f|), on a relative decrease below
  ftol over ``ftol_window`` iterations, or at ``max_iter``.

The paper gives none of these constants; they are this project's reading
(listed with the other readings in the design notes).  Only the converged
point is compared with the GPU solver, never the iterates.

Pins (tests/test_oracle_solvers.py): the two-loop recursion equals the dense
BFGS inverse update applied to gamma*I; returned steps satisfy the strong-Wolfe
conditions; a convex quadratic and Rosenbrock reach their known minimisers;
the result on small RPCA instances matches an independent convex solve
(oracle.convex), the closed form SVT_{lam_l}(X) when lam_s is huge, and
SciPy's L-BFGS-B.
"""
import math

import numpy as np

CONVERGED, FTOL, MAXITER, LINESEARCH_FAILED, NONFINITE = (
    "gtol", "ftol", "maxiter", "linesearch", "nonfinite")


def two_loop(g, S, Y):
    """Return H g for the L-BFGS inverse-Hessian estimate built from pairs (S, Y)."""
    q = g.copy()
    alphas = []
    for s, y in zip(reversed(S), reversed(Y)):
        rho = 1.0 / float(y @ s)
        a = rho * float(s @ q)
        q -= a * y
        alphas.append((a, rho))
    s_new, y_new = S[-1], Y[-1]
    gamma = float(s_new @ y_new) / float(y_new @ y_new)
    r = gamma * q
    for (s, y), (a, rho) in zip(zip(S, Y), reversed(alphas)):
        b = rho * float(y @ r)
        r += (a - b) * s
    return r


def cubic_min(a0, f0, d0, a1, f1, d1):
    """Minimiser of the cubic interpolating (a0,f0,d0) and (a1,f1,d1), or None."""
    if a0 == a1:
        return None
    e1 = d0 + d1 - 3.0 * (f0 - f1) / (a0 - a1)
    disc = e1 * e1 - d0 * d1
    if disc < 0 or not math.isfinite(disc):
        return None
    e2 = math.copysign(math.sqrt(disc), a1 - a0)
    den = d1 - d0 + 2.0 * e2
    if den == 0 or not math.isfinite(den):
        return None
    return a1 - (a1 - a0) * (d1 + e2 - e1) / den


def strong_wolfe(fg, x, f0, g0, d, alpha0, c1=1e-4, c2=0.9, max_evals=40):
    """Bracketing + zoom strong-Wolfe search.  Returns (alpha, f, g, evals, ok)."""
    dphi0 = float(g0 @ d)
    evals = 0

    def phi(a):
        nonlocal evals
        evals += 1
        f, g = fg(x + a * d)
        return f, g, float(g @ d)

    def zoom(lo, hi):
        # lo/hi are tuples (alpha, f, dphi, g); lo satisfies sufficient decrease
        while evals < max_evals:
            a_lo, f_lo, d_lo, _ = lo
            a_hi, f_hi, d_hi, _ = hi
            width = abs(a_hi - a_lo)
            a = cubic_min(a_lo, f_lo, d_lo, a_hi, f_hi, d_hi)
            left, right = min(a_lo, a_hi), max(a_lo, a_hi)
            if a is None or not (left + 0.01 * width <= a <= right - 0.01 * width):
                a = 0.5 * (a_lo + a_hi)
            if width <= 1e-16 * max(1.0, right):
                return lo, False
            f, g, dp = phi(a)
            cur = (a, f, dp, g)
            if not math.isfinite(f):
                hi = cur
                continue
            if f > f0 + c1 * a * dphi0 or f >= f_lo:
                hi = cur
            else:
                if abs(dp) <= -c2 * dphi0:
                    return cur, True
                if dp * (a_hi - a_lo) >= 0:
                    hi = lo
                lo = cur
        return lo, False

    prev = (0.0, f0, dphi0, g0)
    a = alpha0
    i = 1
    while evals < max_evals:
        f, g, dp = phi(a)
        cur = (a, f, dp, g)
        if not math.isfinite(f):
            # step too long: shrink and retry
            a = 0.5 * (prev[0] + a)
            continue
        if f > f0 + c1 * a * dphi0 or (i > 1 and f >= prev[1]):
            res, ok = zoom(prev, cur)
            break
        if abs(dp) <= -c2 * dphi0:
            res, ok = cur, True
            break
        if dp >= 0:
            res, ok = zoom(cur, prev)
            break
        # extrapolate: cubic step clamped to [a + 0.01 (a - a_prev), 10 a]
        a_new = cubic_min(prev[0], prev[1], prev[2], a, f, dp)
        lo_b, hi_b = a + 0.01 * (a - prev[0]), 10.0 * a
        if a_new is None or not (lo_b <= a_new <= hi_b):
            a_new = min(max(2.0 * a, lo_b), hi_b)
        prev = cur
        a = a_new
        i += 1
    else:
        res, ok = prev, False
    alpha, f, _, g = res
    sufficient = alpha > 0 and f <= f0 + c1 * alpha * dphi0
    return alpha, f, g, evals, (ok or sufficient)


def lbfgs(fg, x0, mem=10, max_iter=20000, gtol=1e-10, ftol=1e-15, ftol_window=5,
          c1=1e-4, c2=0.9, callback=None):
    """Minimise fg (returns f, grad) from x0.  Returns dict(x, f, g, iters, evals, status)."""
    x = np.array(x0, dtype=np.float64)
    f, g = fg(x)
    evals = 1
    S, Y = [], []
    fhist = [f]
    status = MAXITER
    it = 0
    reset_once = False
    while it < max_iter:
        if not (math.isfinite(f) and np.all(np.isfinite(g))):
            status = NONFINITE
            break
        if np.max(np.abs(g)) <= gtol * max(1.0, abs(f)):
            status = CONVERGED
            break
        d = -two_loop(g, S, Y) if S else -g
        gtd = float(g @ d)
        if not gtd < 0:
            S, Y = [], []
            d = -g
            gtd = -float(g @ g)
        alpha0 = 1.0 if it > 0 else min(1.0, 1.0 / float(np.sum(np.abs(g))))
        alpha, f_new, g_new, ne, ok = strong_wolfe(fg, x, f, g, d, alpha0, c1, c2)
        evals += ne
        if not ok or alpha == 0:
            if S and not reset_once:
                S, Y = [], []
                reset_once = True
                continue
            status = LINESEARCH_FAILED
            break
        reset_once = False
        s = alpha * d
        y = g_new - g
        sy = float(s @ y)
        if sy > 1e-10 * float(np.linalg.norm(s)) * float(np.linalg.norm(y)):
            S.append(s)
            Y.append(y)
            if len(S) > mem:
                S.pop(0)
                Y.pop(0)
        x = x + s
        f, g = f_new, g_new
        it += 1
        fhist.append(f)
        if callback is not None:
            callback(it, x, f, g)
        if len(fhist) > ftol_window:
            old = fhist[-1 - ftol_window]
            if (old - f) <= ftol * max(1.0, abs(f)):
                status = FTOL
                break
    return dict(x=x, f=f, g=g, iters=it, evals=evals, status=status)
