"""Convergence certificate of Sec. 3.4, FP64 (oracle; test infrastructure only).

Normalised form (Sec. 3.4 sets lam_l = 1 "or absorbs 1/lam_l into phi"):
D = grad phi(L) / lam_l.  With the full SVD L = [U1 U2] diag(Sigma1, 0) [V1 V2]^T
and the subdifferential of the nuclear norm (eq. subdiff), the smallest
element E of d||L||_* + D satisfies

    ||E||_F^2 = ||I + U1^T D V1||^2 + ||U1^T D V2||^2 + ||U2^T D V1||^2
                + min_{||W'|| <= 1} ||U2^T D V2 + W'||^2,

the last term being sum_i (sigma_i(U2^T D V2) - 1)_+^2 (projection onto the
unit spectral-norm ball).  Reading: the paper prints "I - U1^T D V1"; with D =
+grad phi / lam_l and X in d||L||_* equal to U1 V1^T + W, the block is I + U1^T D V1,
which vanishes at a stationary point of f (there D V1 = -U1).  The last term is
sign-symmetric.

The singular vectors of L come from the factors (footnote of Sec. 3.4): QR of
U and V, then an SVD of the small R_U R_V^T.  Numerical rank r counts singular
values above tau * sigma_1; the truncated part adds ||L - L_r||_F / lam_l to
||E||_F (grad phi is 1-Lipschitz, Sec. 3.2).

Gap (eq. Fbound and the bound on ||L - L*||_F that follows it):
F(L) - F* <= ||E||_F * (lam_l ||L||_F + F_bound), F_bound = min(F(L), phi(0), best
F seen) >= F*.  Certified means gap / F(L) <= rel_tol.

Pins (tests/test_oracle_certificate.py): exact and efficient forms agree;
~0 at the convex (FISTA) optimum; the gap bound dominates the true gap
F(L_t) - F* along iterates; at U = V = 0 the value is sum (sigma_i(D) - 1)_+^2
from LAPACK; a positive plateau when k < rank(L*).
"""
import numpy as np

from .objective import grad_phi, phi


def factor_svd(U, V, tau=1e-10):
    """Thin SVD of L = U V^T from the factors.  Returns (U1, sig_r, V1, sig_all)."""
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    Qu, Ru = np.linalg.qr(U)
    Qv, Rv = np.linalg.qr(V)
    Ur, s, Vrt = np.linalg.svd(Ru @ Rv.T)
    if s.size == 0 or s[0] <= 0:
        r = 0
    else:
        r = int(np.count_nonzero(s > tau * s[0]))
    return Qu @ Ur[:, :r], s[:r], Qv @ Vrt.T[:, :r], s


def _terms_exact(D, U1, V1):
    m, n = D.shape
    r = U1.shape[1]
    if r:
        Qu = np.linalg.qr(U1, mode="complete")[0]
        Qv = np.linalg.qr(V1, mode="complete")[0]
        Ut = np.concatenate([U1, Qu[:, r:]], axis=1)
        Vt = np.concatenate([V1, Qv[:, r:]], axis=1)
    else:
        Ut, Vt = np.eye(m), np.eye(n)
    A = Ut.T @ D @ Vt
    T1 = float(np.sum((np.eye(r) + A[:r, :r]) ** 2))
    T2 = float(np.sum(A[:r, r:] ** 2))
    T3 = float(np.sum(A[r:, :r] ** 2))
    sv = np.linalg.svd(A[r:, r:], compute_uv=False)
    T4 = float(np.sum(np.maximum(sv - 1.0, 0.0) ** 2))
    return T1, T2, T3, T4, sv


def _terms_efficient(D, U1, V1):
    r = U1.shape[1]
    DV1 = D @ V1
    DtU1 = D.T @ U1
    C = U1.T @ DV1
    T1 = float(np.sum((np.eye(r) + C) ** 2))
    nC = float(np.sum(C * C))
    T2 = max(float(np.sum(DtU1 * DtU1)) - nC, 0.0)
    T3 = max(float(np.sum(DV1 * DV1)) - nC, 0.0)
    M = D - U1 @ DtU1.T - DV1 @ V1.T + U1 @ C @ V1.T
    sv = np.linalg.svd(M, compute_uv=False)
    T4 = float(np.sum(np.maximum(sv - 1.0, 0.0) ** 2))
    normM2 = float(np.sum(D * D)) - float(np.sum(DtU1 * DtU1)) - float(np.sum(DV1 * DV1)) + nC
    return T1, T2, T3, T4, sv, normM2


def certificate(U, V, X, lam_s, lam_l, mask=None, tau=1e-10, F_best=None,
                form="exact", rel_tol=1e-3, mu=0.0):
    """Certificate terms, F(L), F_bound and the gap bound at L = U V^T."""
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    X = np.asarray(X, np.float64)
    L = U @ V.T
    D = grad_phi(L, X, lam_s, mask, mu) / lam_l
    U1, sig, V1, sig_all = factor_svd(U, V, tau)
    r = sig.size
    if form == "exact":
        T1, T2, T3, T4, sv = _terms_exact(D, U1, V1)
        normM2 = float(np.sum(sv * sv))
    else:
        T1, T2, T3, T4, sv, normM2 = _terms_efficient(D, U1, V1)
    trunc = float(np.sqrt(np.sum(sig_all[r:] ** 2))) / lam_l
    E = float(np.sqrt(max(T1 + T2 + T3 + T4, 0.0))) + trunc
    phiL = phi(L, X, lam_s, mask, mu)
    F = lam_l * float(np.sum(sig_all)) + phiL
    phi0 = phi(np.zeros_like(X), X, lam_s, mask, mu)
    F_bound = min(F, phi0) if F_best is None else min(F, phi0, F_best)
    normL = float(np.sqrt(np.sum(sig_all ** 2)))
    gap = E * (lam_l * normL + F_bound)
    rel_gap = gap / F if F > 0 else (0.0 if gap == 0 else np.inf)
    return dict(T1=T1, T2=T2, T3=T3, T4=T4, r=r, sigma=sig_all, E=E, F=F, phi=phiL,
                phi0=phi0, F_bound=F_bound, normL=normL, gap=gap, rel_gap=rel_gap,
                certified=bool(rel_gap <= rel_tol), sv_perp=sv, normM2=normM2,
                trunc=trunc)
