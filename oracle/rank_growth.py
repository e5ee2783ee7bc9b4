"""Rank growth of the factorisation (Sec. 4.1), FP64 (oracle; test
infrastructure only).

Sec. 4.1 grows k on the fly: after the solver stops, one column is added to U
and V, L <- L + u v^T, and kept when it lowers the objective.  The paper leaves
the column open; the reading here takes the direction the certificate of
Sec. 3.4 already measures.  With D = grad phi(L) / lam_l and the projections
P_U^perp, P_V^perp onto the complements of L's column and row spaces, let
(sigma, u, v) be the top singular triplet of M = P_U^perp D P_V^perp.  L is
optimal for the convex problem only if sigma <= 1 (the last block of the
certificate).  Along Delta = -t u v^T (t >= 0; u, v orthogonal to L's spaces):

  * the nuclear norm grows by exactly t, and the factored regulariser of the
    balanced column pair (sqrt(t) u, -sqrt(t) v) is lam_l t as well;
  * <grad phi, Delta> = -t lam_l u^T D v = -t lam_l sigma;
  * phi's curvature along a unit-Frobenius direction is at most 1 (the Huber
    function's second derivative is 0 or 1; unobserved entries add nothing), so
    phi(L + Delta) <= phi(L) - t lam_l sigma + t^2 / 2.

Hence f(t) <= f(0) - t lam_l (sigma - 1) + t^2 / 2, minimised at
t = lam_l (sigma - 1): the grown factors [U, sqrt(t) u], [V, -sqrt(t) v] lower
f by at least lam_l^2 (sigma - 1)^2 / 2 whenever sigma > 1.

Pins (tests/test_oracle_rank_growth.py): the decrease bound on random and
stationary points; the directional derivative of f along the pair matches
lam_l (1 - sigma) by central differences; sigma agrees with the certificate's
last block (its (sigma - 1)_+^2 term); sigma <= 1 at a certified optimum and
> 1 at a stationary point whose rank bound is below rank(L*).
"""
import numpy as np

from .certificate import factor_svd
from .objective import grad_phi


def growth_direction(U, V, X, lam_s, lam_l, mask=None, tau=1e-10):
    """Top singular triplet of P_U^perp D P_V^perp at L = U V^T.
    Returns (sigma, u, v) with u^T D v = sigma >= 0 (u: m, v: n, unit norm)."""
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    D = grad_phi(U @ V.T, np.asarray(X, np.float64), lam_s, mask) / lam_l
    U1, _, V1, _ = factor_svd(U, V, tau)
    M = D - U1 @ (U1.T @ D)
    M = M - (M @ V1) @ V1.T
    Us, s, Vt = np.linalg.svd(M, full_matrices=False)
    u, v = Us[:, 0], Vt[0]
    if u @ D @ v < 0:
        u, v = -u, -v
    return float(s[0]), u, v


def grow(U, V, X, lam_s, lam_l, mask=None):
    """One growth step: returns (U', V', sigma, t).  When sigma <= 1 the factors
    come back unchanged (t = 0)."""
    sigma, u, v = growth_direction(U, V, X, lam_s, lam_l, mask)
    if sigma <= 1.0:
        return np.asarray(U, np.float64), np.asarray(V, np.float64), sigma, 0.0
    t = lam_l * (sigma - 1.0)
    Un = np.concatenate([np.asarray(U, np.float64), np.sqrt(t) * u[:, None]], axis=1)
    Vn = np.concatenate([np.asarray(V, np.float64), -np.sqrt(t) * v[:, None]], axis=1)
    return Un, Vn, sigma, t


def decrease_bound(sigma, lam_l):
    """Guaranteed decrease of f by one growth step."""
    return 0.5 * (lam_l * max(sigma - 1.0, 0.0)) ** 2
