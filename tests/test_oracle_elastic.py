"""Pins for the elastic-net marginal in oracle.objective (Sec. 1: other
regularisers r(S) marginalise the same way; r(S) = lam_s ||S||_1 + mu/2 ||S||_F^2).

* per entry, rho(r) equals a brute-force minimisation over s of
  1/2 (r + s)^2 + lam |s| + mu/2 s^2 (dense grid refined by golden section), and
  rho' equals its central difference;
* mu = 0 is the Huber function exactly; mu -> infinity tends to r^2/2 (S forced to 0);
* phi(L) equals the brute-force joint minimisation over S (bound-constrained
  solver on a tiny matrix), and the factored gradient matches central differences;
* sparse_part is the minimiser: its objective equals phi;
* the convex optimum from FISTA-SVT (elastic phi) and the factored L-BFGS optimum
  agree (k > rank(L*)), and the certificate certifies it.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import certificate as ce
from oracle import convex as cv
from oracle import lbfgs as lb
from oracle import objective as ob
from oracle import rsvd as rs
from paper_1702_02241_amd import synth


def _brute(r, lam, mu):
    def g(s):
        return 0.5 * (r + s) ** 2 + lam * abs(s) + 0.5 * mu * s * s
    grid = np.linspace(-abs(r) - 1, abs(r) + 1, 4001)
    vals = 0.5 * (r + grid) ** 2 + lam * np.abs(grid) + 0.5 * mu * grid ** 2
    b = grid[int(np.argmin(vals))]
    lo, hi = b - 1e-3 * (abs(r) + 1), b + 1e-3 * (abs(r) + 1)
    gr = (np.sqrt(5) - 1) / 2
    for _ in range(100):
        a1 = hi - gr * (hi - lo)
        b1 = lo + gr * (hi - lo)
        if g(a1) < g(b1):
            hi = b1
        else:
            lo = a1
    return g(0.5 * (lo + hi))


@pytest.mark.parametrize("mu", [0.0, 0.3, 2.0])
def test_entry_marginal_is_the_brute_force_minimum(mu):
    lam = 0.7
    for r in np.linspace(-4, 4, 41):
        assert abs(ob.huber(r, lam, mu) - _brute(r, lam, mu)) <= 1e-9 * max(1.0, abs(r) ** 2)
        h = 1e-6
        d = (ob.huber(r + h, lam, mu) - ob.huber(r - h, lam, mu)) / (2 * h)
        assert abs(d - ob.huber_deriv(r, lam, mu)) <= 1e-6


def test_limits_in_mu():
    r = np.linspace(-5, 5, 101)
    assert np.array_equal(ob.huber(r, 0.5, 0.0), ob.huber(r, 0.5))
    assert np.array_equal(ob.huber_deriv(r, 0.5, 0.0), np.clip(r, -0.5, 0.5))
    big = ob.huber(r, 0.5, 1e12)
    assert np.allclose(big, 0.5 * r * r, rtol=1e-9, atol=1e-9)
    assert np.allclose(ob.huber_deriv(r, 0.5, 1e12), r, rtol=1e-9, atol=1e-9)


def test_phi_is_the_joint_minimum_and_sparse_part_attains_it():
    rng = np.random.default_rng(31)
    m, n, lam, mu = 4, 3, 0.4, 0.8
    X = rng.normal(size=(m, n)) * 2
    L = rng.normal(size=(m, n))
    mask = (rng.random((m, n)) < 0.75).astype(np.uint8)
    W = mask.astype(np.float64)

    def obj(s):
        S = s.reshape(m, n)
        return 0.5 * np.sum((W * (L + S - X)) ** 2) + lam * np.sum(np.abs(S)) + 0.5 * mu * np.sum(S * S)

    best = min(minimize(obj, x0, method="Powell", options=dict(xtol=1e-12, ftol=1e-14, maxiter=200000)).fun
               for x0 in (np.zeros(m * n), rng.normal(size=m * n)))
    ph = ob.phi(L, X, lam, mask, mu)
    assert abs(ph - best) <= 1e-7 * max(1.0, best)
    S = ob.sparse_part(L, X, lam, mask, mu)
    assert abs(obj(S.ravel()) - ph) <= 1e-12 * max(1.0, ph)


def test_factored_gradient_matches_central_differences():
    rng = np.random.default_rng(32)
    m, n, k, lam_s, lam_l, mu = 9, 7, 3, 0.3, 0.6, 1.5
    X = rng.normal(size=(m, n)) * 2
    U = rng.normal(size=(m, k))
    V = rng.normal(size=(n, k))
    f, gU, gV = ob.objgrad(U, V, X, lam_s, lam_l, mu=mu)
    h = 1e-6
    for (i, j) in [(0, 0), (4, 2), (8, 1)]:
        Up, Um = U.copy(), U.copy()
        Up[i, j] += h
        Um[i, j] -= h
        d = (ob.objective(Up, V, X, lam_s, lam_l, mu=mu) - ob.objective(Um, V, X, lam_s, lam_l, mu=mu)) / (2 * h)
        assert abs(d - gU[i, j]) <= 1e-6 * max(1.0, abs(d))
    for (i, j) in [(0, 0), (6, 2)]:
        Vp, Vm = V.copy(), V.copy()
        Vp[i, j] += h
        Vm[i, j] -= h
        d = (ob.objective(U, Vp, X, lam_s, lam_l, mu=mu) - ob.objective(U, Vm, X, lam_s, lam_l, mu=mu)) / (2 * h)
        assert abs(d - gV[i, j]) <= 1e-6 * max(1.0, abs(d))


def test_factored_and_convex_optima_agree_and_certify():
    p = synth.gaussian_rpca(m=60, n=45, r=3, k=6, seed=33, lam_s=0.3, lam_l=4.0)
    mu = 0.2  # rank(L*) = 5 here; the l1 optimum has rank 3
    cvx = cv.fista_svt(p.X, p.lam_s, p.lam_l, max_iter=20000, tol=1e-13, mu=mu)
    assert cvx["rank"] < 6
    Om = synth.gaussian_matrix(p.n, 16, 34)
    U0, V0 = rs.rsvd_factors(p.X, 6, Om)
    res = lb.lbfgs(ob.make_fg(p.X, p.lam_s, p.lam_l, 6, mu=mu), ob.pack(U0, V0))
    U, V = ob.unpack(res["x"], p.m, p.n, 6)
    F = ob.convex_objective(U @ V.T, p.X, p.lam_s, p.lam_l, mu=mu)
    c = ce.certificate(U, V, p.X, p.lam_s, p.lam_l, mu=mu)
    # the elastic-net optimum differs from the l1 one
    F_l1 = cv.fista_svt(p.X, p.lam_s, p.lam_l, max_iter=20000, tol=1e-13)["F"]
    print("F factored", F, "F convex", cvx["F"], "rel_gap", c["rel_gap"], "l1 F", F_l1)
    assert abs(F - cvx["F"]) <= 1e-8 * cvx["F"]
    assert c["rel_gap"] <= 1e-6
    assert abs(F_l1 - cvx["F"]) > 1e-3 * cvx["F"]
