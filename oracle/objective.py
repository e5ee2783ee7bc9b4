"""Split-SPCP objective and gradient in FP64 (oracle; test infrastructure only).

Definitions (Sec. 1 "Marginalization in S", eq. PhiDef; Sec. 5 eq. Thm5):

    phi(L)  = min_S 1/2 ||P_Omega(L + S - X)||_F^2 + lam_s ||S||_1
            = sum over observed (i,j) of rho_{lam_s}(L_ij - X_ij)
    f(U,V)  = phi(U V^T) + lam_l/2 (||U||_F^2 + ||V||_F^2)          (eq. smoothNC)

rho is the Huber function: per entry the minimiser over s of
1/2 (r + s)^2 + lam |s| is s* = -soft(r, lam), which leaves r + s* = clip(r, -lam, lam)
and the value r^2/2 for |r| <= lam, lam|r| - lam^2/2 otherwise.  Entries outside
Omega carry no loss, so their optimal s is 0 and they add nothing.

Gradient (Sec. 3.2 eq. diff): grad phi(L) = P_Omega(L + S* - X) = P_Omega(clip(L - X)),
so with G = Omega .* clip(U V^T - X, -lam_s, lam_s):
    d f / dU = G V + lam_l U,     d f / dV = G^T U + lam_l V.

Elastic net (Sec. 1 lists it among the regularisers r(S) that marginalise):
with r(S) = lam_s ||S||_1 + mu/2 ||S||_F^2 (Zou & Hastie 2005) the per-entry
minimiser over s of 1/2 (r + s)^2 + lam |s| + mu/2 s^2 is s* = -soft(r, lam)/(1 + mu),
which leaves rho(r) = r^2/2 for |r| <= lam and lam|r| - lam^2/2 + kappa/2 (|r| - lam)^2
otherwise, kappa = mu/(1 + mu); rho'(r) = c + kappa (r - c) with c = clip(r, -lam, lam).
mu = 0 (the default everywhere) is the l1 case above; rho' stays 1-Lipschitz.

Pins (tests/test_oracle_objective.py, tests/test_oracle_elastic.py): brute-force
minimisation over S on tiny inputs (per-entry grid + golden section, and a joint
bound-constrained solve), central finite differences of f, midpoint convexity of
phi (Lemma 1), invariance f(UQ, VQ) = f(U, V) for orthogonal Q (Theorem 1); for
the elastic net the same brute-force and difference checks, mu = 0 giving the
Huber function and mu -> infinity the plain quadratic.
"""
import numpy as np


def kappa_of(mu):
    """Slope of rho' beyond the threshold for the elastic net weight mu."""
    return mu / (1.0 + mu)


def huber(r, lam, mu=0.0):
    """rho_lam(r): r^2/2 if |r| <= lam else lam|r| - lam^2/2 (+ kappa/2 (|r| - lam)^2 for
    the elastic net); tie -> quadratic branch."""
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(r)
    b = a - lam
    return np.where(a <= lam, 0.5 * r * r, lam * a - 0.5 * lam * lam + 0.5 * kappa_of(mu) * b * b)


def huber_deriv(r, lam, mu=0.0):
    """rho_lam'(r) = clip(r, -lam, lam) (+ kappa (r - clip) for the elastic net)."""
    r = np.asarray(r, dtype=np.float64)
    c = np.clip(r, -lam, lam)
    return c + kappa_of(mu) * (r - c) if mu else c


def soft(r, lam):
    """Soft threshold (the prox of lam|.|)."""
    r = np.asarray(r, dtype=np.float64)
    return np.sign(r) * np.maximum(np.abs(r) - lam, 0.0)


def _omega(mask, shape):
    if mask is None:
        return np.ones(shape, dtype=np.float64)
    return (np.asarray(mask) != 0).astype(np.float64)


def phi(L, X, lam_s, mask=None, mu=0.0):
    """Marginal phi(L) = sum over Omega of rho_{lam_s}(L - X)."""
    W = _omega(mask, X.shape)
    return float(np.sum(W * huber(np.asarray(L, np.float64) - X, lam_s, mu)))


def grad_phi(L, X, lam_s, mask=None, mu=0.0):
    """grad phi(L) = Omega .* rho'(L - X) (= clip(L - X, -lam_s, lam_s) for mu = 0)."""
    W = _omega(mask, X.shape)
    return W * huber_deriv(np.asarray(L, np.float64) - X, lam_s, mu)


def sparse_part(L, X, lam_s, mask=None, mu=0.0):
    """The marginalised S*: Omega .* soft(X - L, lam_s) / (1 + mu) (zero where unobserved)."""
    W = _omega(mask, X.shape)
    return W * soft(X - np.asarray(L, np.float64), lam_s) / (1.0 + mu)


def objective(U, V, X, lam_s, lam_l, mask=None, mu=0.0):
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    return phi(U @ V.T, X, lam_s, mask, mu) + 0.5 * lam_l * (np.sum(U * U) + np.sum(V * V))


def objgrad(U, V, X, lam_s, lam_l, mask=None, mu=0.0):
    """Return (f, dF/dU, dF/dV) at (U, V), all FP64."""
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    X = np.asarray(X, np.float64)
    R = U @ V.T - X
    W = _omega(mask, X.shape)
    f = float(np.sum(W * huber(R, lam_s, mu))) + 0.5 * lam_l * (np.sum(U * U) + np.sum(V * V))
    G = W * huber_deriv(R, lam_s, mu)
    gU = G @ V + lam_l * U
    gV = G.T @ U + lam_l * V
    return f, gU, gV


def convex_objective(L, X, lam_s, lam_l, mask=None, mu=0.0):
    """F(L) = lam_l ||L||_* + phi(L)  (eq. genConvex)."""
    s = np.linalg.svd(np.asarray(L, np.float64), compute_uv=False)
    return lam_l * float(np.sum(s)) + phi(L, X, lam_s, mask, mu)


def pack(U, V):
    """Flatten (U, V) into one vector x = [vec_rows(U); vec_rows(V)]."""
    return np.concatenate([np.asarray(U, np.float64).ravel(), np.asarray(V, np.float64).ravel()])


def unpack(x, m, n, k):
    return x[: m * k].reshape(m, k), x[m * k:].reshape(n, k)


def make_fg(X, lam_s, lam_l, k, mask=None, mu=0.0):
    """Objective on the flat vector x, as used by the L-BFGS oracle."""
    m, n = X.shape

    def fg(x):
        U, V = unpack(x, m, n, k)
        f, gU, gV = objgrad(U, V, X, lam_s, lam_l, mask, mu)
        return f, pack(gU, gV)

    return fg
