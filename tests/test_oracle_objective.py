"""Pins for oracle.objective: the Huber marginalisation identity and the gradient.

Each check is independent of the formula it tests: phi is compared with a
brute-force minimisation over S (Sec. 1 eq. PhiDef, Sec. 5 eq. Thm5), the
gradient with finite differences, plus invariants from Lemma 1 (convexity
of phi) and Theorem 1 (f(UQ, VQ) = f(U, V)).
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import objective as ob


def _golden(fun, lo, hi, iters=200):
    g = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = lo, hi
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = fun(c), fun(d)
    for _ in range(iters):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = fun(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = fun(d)
    x = 0.5 * (a + b)
    return fun(x)


def _phi_brute_entrywise(L, X, lam, mask=None):
    """min over S of 1/2||P(L+S-X)||^2 + lam||S||_1, entry by entry (dense grid + golden section)."""
    total = 0.0
    for (i, j), r in np.ndenumerate(L - X):
        if mask is not None and not mask[i, j]:
            # no loss term: the minimiser is s = 0 and the entry adds nothing
            fun = lambda s: lam * abs(s)  # noqa: E731
        else:
            fun = lambda s, r=r: 0.5 * (r + s) ** 2 + lam * abs(s)  # noqa: E731
        span = abs(r) + 1.0
        grid = np.linspace(-span, span, 100001)
        vals = np.array([fun(s) for s in grid[::1000]])  # coarse pass to bracket
        fine = 0.5 * (grid[:-1:1000] + grid[1::1000])
        del fine
        s0 = grid[::1000][int(np.argmin(vals))]
        h = 2.0 * span / 100.0
        dense = np.linspace(s0 - h, s0 + h, 1001)
        dv = np.array([fun(s) for s in dense])
        s1 = dense[int(np.argmin(dv))]
        step = dense[1] - dense[0]
        total += _golden(fun, s1 - step, s1 + step)
    return total


def _phi_brute_joint(L, X, lam, mask=None):
    """Joint bound-constrained solve with S = P - N, P, N >= 0 (smooth QP)."""
    R = (L - X).ravel()
    W = np.ones_like(R) if mask is None else (mask.ravel() != 0).astype(float)
    nvar = R.size

    def fun(z):
        P, N = z[:nvar], z[nvar:]
        res = W * (R + P - N)
        val = 0.5 * res @ res + lam * (P.sum() + N.sum())
        g = W * res
        return val, np.concatenate([g + lam, -g + lam])

    out = minimize(fun, np.zeros(2 * nvar), jac=True, method="L-BFGS-B",
                   bounds=[(0, None)] * (2 * nvar), options=dict(ftol=1e-16, gtol=1e-13, maxiter=10000))
    return out.fun


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_phi_matches_brute_force_minimisation_over_S(seed):
    rng = np.random.default_rng(seed)
    L = rng.normal(size=(4, 3))
    X = rng.normal(size=(4, 3)) * 2.0
    lam = 0.7
    closed = ob.phi(L, X, lam)
    brute = _phi_brute_entrywise(L, X, lam)
    joint = _phi_brute_joint(L, X, lam)
    print(f"phi closed={closed:.15f} entrywise={brute:.15f} joint={joint:.15f}")
    assert abs(closed - brute) <= 1e-12
    assert abs(closed - joint) <= 1e-8


def test_phi_masked_brute_force():
    rng = np.random.default_rng(7)
    L = rng.normal(size=(4, 3))
    X = rng.normal(size=(4, 3)) * 2.0
    mask = (rng.random((4, 3)) < 0.6).astype(np.uint8)
    lam = 0.4
    closed = ob.phi(L, X, lam, mask)
    brute = _phi_brute_entrywise(L, X, lam, mask)
    print(f"masked phi closed={closed:.15f} brute={brute:.15f}")
    assert abs(closed - brute) <= 1e-12


def test_sparse_part_is_the_minimiser():
    rng = np.random.default_rng(3)
    L = rng.normal(size=(5, 4))
    X = rng.normal(size=(5, 4)) * 3.0
    lam = 0.5
    S = ob.sparse_part(L, X, lam)
    val = 0.5 * np.sum((L + S - X) ** 2) + lam * np.sum(np.abs(S))
    assert abs(val - ob.phi(L, X, lam)) <= 1e-12
    # any perturbation of S does not decrease the value
    for _ in range(20):
        S2 = S + 1e-3 * rng.normal(size=S.shape)
        val2 = 0.5 * np.sum((L + S2 - X) ** 2) + lam * np.sum(np.abs(S2))
        assert val2 >= val - 1e-15


def test_huber_reduces_to_least_squares_for_large_lambda():
    rng = np.random.default_rng(4)
    R = rng.normal(size=(6, 5))
    assert np.allclose(ob.huber(R, 1e6), 0.5 * R * R, rtol=0, atol=0)
    # and to lam|r| - lam^2/2 (an l1 fit) in the linear regime
    lam = 1e-3
    big = R[np.abs(R) > lam]
    assert np.allclose(ob.huber(big, lam), lam * np.abs(big) - 0.5 * lam * lam)


def test_gradient_matches_central_finite_differences():
    rng = np.random.default_rng(5)
    m, n, k = 6, 5, 3
    U = rng.normal(size=(m, k))
    V = rng.normal(size=(n, k))
    X = rng.normal(size=(m, n)) * 2
    lam_s, lam_l = 0.8, 0.3
    h = 1e-6
    # keep every residual at least 10h away from the kink |r| = lam_s
    R = U @ V.T - X
    near = np.abs(np.abs(R) - lam_s) < 1e-3
    X[near] += 0.01
    f, gU, gV = ob.objgrad(U, V, X, lam_s, lam_l)
    g = ob.pack(gU, gV)
    x = ob.pack(U, V)
    fd = np.empty_like(x)
    for i in range(x.size):
        e = np.zeros_like(x)
        e[i] = h
        Up, Vp = ob.unpack(x + e, m, n, k)
        Um, Vm = ob.unpack(x - e, m, n, k)
        fd[i] = (ob.objective(Up, Vp, X, lam_s, lam_l) - ob.objective(Um, Vm, X, lam_s, lam_l)) / (2 * h)
    rel = np.linalg.norm(fd - g) / np.linalg.norm(g)
    print(f"FD gradient relative error {rel:.3e}")
    assert rel <= 1e-6


def test_masked_gradient_ignores_unobserved_entries():
    rng = np.random.default_rng(6)
    m, n, k = 7, 6, 2
    U, V = rng.normal(size=(m, k)), rng.normal(size=(n, k))
    X = rng.normal(size=(m, n))
    mask = (rng.random((m, n)) < 0.5).astype(np.uint8)
    f1, gU1, gV1 = ob.objgrad(U, V, X, 0.3, 0.2, mask)
    X2 = X + (1 - mask) * rng.normal(size=(m, n)) * 100
    f2, gU2, gV2 = ob.objgrad(U, V, X2, 0.3, 0.2, mask)
    assert f1 == f2 and np.array_equal(gU1, gU2) and np.array_equal(gV1, gV2)


def test_phi_is_convex_along_random_lines():
    # Lemma 1: the marginal of a jointly convex function is convex
    rng = np.random.default_rng(8)
    X = rng.normal(size=(8, 6)) * 3
    for _ in range(50):
        A, B = rng.normal(size=(8, 6)) * 2, rng.normal(size=(8, 6)) * 2
        t = rng.random()
        lhs = ob.phi(t * A + (1 - t) * B, X, 0.5)
        rhs = t * ob.phi(A, X, 0.5) + (1 - t) * ob.phi(B, X, 0.5)
        assert lhs <= rhs + 1e-12


def test_objective_invariant_under_orthogonal_rotation():
    # Theorem 1 / its proof: (U, V) -> (U Q, V Q) leaves U V^T and the norms unchanged
    rng = np.random.default_rng(9)
    U, V = rng.normal(size=(9, 4)), rng.normal(size=(7, 4))
    X = rng.normal(size=(9, 7))
    Q = np.linalg.qr(rng.normal(size=(4, 4)))[0]
    f1 = ob.objective(U, V, X, 0.3, 0.7)
    f2 = ob.objective(U @ Q, V @ Q, X, 0.3, 0.7)
    assert abs(f1 - f2) <= 1e-12 * abs(f1)
