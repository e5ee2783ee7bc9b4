"""Randomized-SVD initialisation of the factors, FP64 (oracle; tests only).

Sec. 4.2: start from U0 = U_k Sigma_k^{1/2}, V0 = V_k Sigma_k^{1/2} where the
rank-k SVD of A*(X) (the zero-filled sampled data) is approximated by a
randomized SVD.  The randomized SVD follows Halko, Martinsson & Tropp
(randomized subspace iteration): Y = A Omega_s with an n x (k + p) Gaussian
test matrix, q power steps with re-orthonormalisation after every product,
B = Q^T A, small SVD of B.  The test matrix is an input (drawn by the
caller), so the GPU path and this oracle see the same random numbers.
Orthonormalisation here is Householder QR (numpy), independent of whatever
the GPU uses.

Reading: no 1/p rescaling of A*(X) for partial observation (the text takes
the SVD of A*(X) as is); p and q are parameters (defaults 10 and 2).

Pins: with q large or an exactly rank-k input, the result equals the
truncated LAPACK SVD (U0 V0^T = best rank-k approximation).
"""
import numpy as np


def rsvd_factors(X, k, Omega, q=2, mask=None):
    """Return (U0, V0) with U0 V0^T ~ best rank-k approximation of P_Omega(X)."""
    A = np.asarray(X, np.float64)
    if mask is not None:
        A = A * (np.asarray(mask) != 0)
    Om = np.asarray(Omega, np.float64)
    Q = np.linalg.qr(A @ Om)[0]
    for _ in range(q):
        Z = np.linalg.qr(A.T @ Q)[0]
        Q = np.linalg.qr(A @ Z)[0]
    B = Q.T @ A
    Ub, s, Vbt = np.linalg.svd(B, full_matrices=False)
    root = np.sqrt(s[:k])
    return (Q @ Ub[:, :k]) * root, Vbt[:k].T * root
