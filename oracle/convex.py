"""Convex reference solve of eq. genConvex by FISTA + SVT (oracle; tests only).

F(L) = lam_l ||L||_* + phi(L).  Sec. 1 notes that proximal gradient methods
apply to this problem; Sec. 3.2 (Moreau-envelope proposition, Combettes
Prop. 12.29) gives that grad phi is 1-Lipschitz, so the step size is 1 and
the proximal step is singular-value soft-thresholding at lam_l computed with a
LAPACK SVD.  Acceleration is FISTA (Beck & Teboulle) with the function-value
adaptive restart of O'Donoghue & Candes.  This solver is independent of the
factored problem: it never forms U or V, so agreement with the L-BFGS oracle
on the factored problem pins both (Theorem 1: local minima of the factored
problem are minima of the rank-constrained problem; with k > rank(L*) that
is the convex optimum).

Pins: the lam_s -> infinity special case (phi = 1/2||L - X||^2) where the
minimiser is exactly SVT_{lam_l}(X); the zero-solution threshold
lam_l >= ||grad phi(0)||_2 <=> L* = 0.
"""
import numpy as np

from .objective import grad_phi, phi


def svt(Z, tau):
    """Singular-value soft threshold: argmin_L tau||L||_* + 1/2||L - Z||_F^2."""
    U, s, Vt = np.linalg.svd(Z, full_matrices=False)
    s = np.maximum(s - tau, 0.0)
    r = int(np.count_nonzero(s))
    return (U[:, :r] * s[:r]) @ Vt[:r], s[:r]


def objective(L, X, lam_s, lam_l, mask=None, sing=None, mu=0.0):
    if sing is None:
        sing = np.linalg.svd(L, compute_uv=False)
    return lam_l * float(np.sum(sing)) + phi(L, X, lam_s, mask, mu)


def fista_svt(X, lam_s, lam_l, mask=None, L0=None, max_iter=20000, tol=1e-13,
              callback=None, mu=0.0):
    """Minimise F(L) by accelerated proximal gradient, step 1.

    Stops when ||L_{t+1} - L_t||_F <= tol * max(1, ||L_t||_F).
    Returns dict(L, F, iters, rank).
    """
    X = np.asarray(X, np.float64)
    L = np.zeros_like(X) if L0 is None else np.array(L0, np.float64)
    Yk = L.copy()
    t = 1.0
    F_prev = objective(L, X, lam_s, lam_l, mask, mu=mu)
    it = 0
    for it in range(1, max_iter + 1):
        L_new, s_new = svt(Yk - grad_phi(Yk, X, lam_s, mask, mu), lam_l)
        F_new = lam_l * float(np.sum(s_new)) + phi(L_new, X, lam_s, mask, mu)
        if F_new > F_prev:
            # adaptive restart: drop the momentum and take a plain step from L
            t = 1.0
            L_new, s_new = svt(L - grad_phi(L, X, lam_s, mask, mu), lam_l)
            F_new = lam_l * float(np.sum(s_new)) + phi(L_new, X, lam_s, mask, mu)
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        step = np.linalg.norm(L_new - L)
        Yk = L_new + ((t - 1.0) / t_new) * (L_new - L)
        done = step <= tol * max(1.0, np.linalg.norm(L))
        L, t, F_prev = L_new, t_new, F_new
        if callback is not None:
            callback(it, L, F_new)
        if done:
            break
    return dict(L=L, F=F_prev, iters=it, rank=int(np.linalg.matrix_rank(L)))
