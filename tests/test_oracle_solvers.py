"""Pins for oracle.lbfgs, oracle.convex, oracle.rsvd on problems with known answers.

* the two-loop recursion equals the dense BFGS inverse update; strong-Wolfe
  conditions hold at returned steps; a convex quadratic is solved;
* Rosenbrock's known minimiser;
* lam_s -> infinity: phi = 1/2||L - X||^2 and the convex minimiser is the
  singular-value soft threshold of X (closed form via LAPACK);
* lam_l >= ||clip(X)||_2 gives L* = 0 (zero-solution threshold);
* the factored L-BFGS solve agrees with the independent FISTA-SVT solve on
  the 256 x 200 Gaussian workload (Theorem 1 with k > rank(L*));
* SciPy's L-BFGS-B reaches the same objective;
* at the solution the factors are balanced, U^T U = V^T V.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import convex as cv
from oracle import lbfgs as lb
from oracle import objective as ob
from oracle import rsvd as rs
from paper_1702_02241_amd import synth


def test_two_loop_equals_dense_bfgs_inverse_update():
    # the two-loop recursion applies the BFGS inverse update (Nocedal & Wright
    # eq. 6.17) m times to H0 = gamma I; build that matrix densely and compare
    rng = np.random.default_rng(0)
    dim, mem = 9, 5
    A = rng.normal(size=(dim, dim))
    H = A @ A.T + np.eye(dim)
    S = [rng.normal(size=dim) for _ in range(mem)]
    Y = [H @ s for s in S]
    gamma = S[-1] @ Y[-1] / (Y[-1] @ Y[-1])
    Hk = gamma * np.eye(dim)
    for s, y in zip(S, Y):
        rho = 1.0 / (y @ s)
        Vm = np.eye(dim) - rho * np.outer(y, s)
        Hk = Vm.T @ Hk @ Vm + rho * np.outer(s, s)
    g = rng.normal(size=dim)
    assert np.allclose(lb.two_loop(g, S, Y), Hk @ g, rtol=1e-12, atol=1e-12)
    # secant condition for the newest pair
    assert np.allclose(lb.two_loop(Y[-1], S, Y), S[-1], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("shift", [0.3, 3.0, 30.0])
def test_strong_wolfe_conditions_hold(shift):
    # phi(a) = f(x + a d) for a smooth non-quadratic 1-D-in-effect function
    def fg(x):
        z = x - shift
        return float(np.sum(np.logaddexp(z, -z) + 0.05 * z ** 4)), np.tanh(z) + 0.2 * z ** 3

    x = np.zeros(4)
    f0, g0 = fg(x)
    d = -g0
    for a0 in (1e-3, 1.0, 50.0):
        a, f, g, ev, ok = lb.strong_wolfe(fg, x, f0, g0, d, a0, c1=1e-4, c2=0.9)
        assert ok
        assert f <= f0 + 1e-4 * a * (g0 @ d)
        assert abs(g @ d) <= 0.9 * abs(g0 @ d)


def test_lbfgs_quadratic_converges_to_solution():
    rng = np.random.default_rng(0)
    dim = 30
    A = rng.normal(size=(dim, dim))
    H = A @ A.T + np.eye(dim)
    b = rng.normal(size=dim)

    def fg(x):
        return 0.5 * x @ H @ x - b @ x, H @ x - b

    # gtol well above the point where f-differences drown in rounding
    res = lb.lbfgs(fg, np.zeros(dim), mem=10, gtol=1e-7, ftol=0)
    print("quadratic iters", res["iters"], res["status"])
    assert res["status"] == lb.CONVERGED
    assert np.allclose(res["x"], np.linalg.solve(H, b), atol=1e-6)


def test_lbfgs_rosenbrock():
    def fg(x):
        a, b = x
        f = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        return f, np.array([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)])

    res = lb.lbfgs(fg, np.array([-1.2, 1.0]), gtol=1e-12, ftol=0)
    assert np.allclose(res["x"], [1.0, 1.0], atol=1e-8)


def _solve_factored(p, k, init_seed=11):
    Om = synth.gaussian_matrix(p.n, k + 10, init_seed)
    U0, V0 = rs.rsvd_factors(p.X, k, Om, mask=p.mask)
    res = lb.lbfgs(ob.make_fg(p.X, p.lam_s, p.lam_l, k, p.mask), ob.pack(U0, V0))
    U, V = ob.unpack(res["x"], p.m, p.n, k)
    return U, V, res


def test_large_lambda_s_gives_svt_closed_form():
    rng = np.random.default_rng(1)
    m, n = 40, 30
    X = rng.normal(size=(m, 4)) @ rng.normal(size=(4, n)) + 0.3 * rng.normal(size=(m, n))
    lam_l = 3.0
    p = synth.Problem(X=X, lam_s=1e6, lam_l=lam_l, k=12)
    U, V, res = _solve_factored(p, 12)
    L_svt, s = cv.svt(X, lam_l)
    rel = np.linalg.norm(U @ V.T - L_svt) / np.linalg.norm(L_svt)
    print("SVT closed form rel err", rel, "rank", s.size, res["status"], res["iters"])
    assert rel <= 1e-8


def test_zero_solution_threshold():
    rng = np.random.default_rng(2)
    m, n, k = 30, 20, 5
    X = rng.normal(size=(m, n))
    lam_s = 0.5
    thresh = np.linalg.norm(np.clip(X, -lam_s, lam_s), 2)
    # above the threshold the minimiser is 0 ...
    res = cv.fista_svt(X, lam_s, 1.01 * thresh, max_iter=200)
    assert np.linalg.norm(res["L"]) == 0.0
    U0, V0 = synth.random_factors(m, n, k, 3, scale=0.1)
    out = lb.lbfgs(ob.make_fg(X, lam_s, 1.01 * thresh, k), ob.pack(U0, V0))
    U, V = ob.unpack(out["x"], m, n, k)
    assert np.linalg.norm(U @ V.T) <= 1e-6
    # ... and below it it is not
    res = cv.fista_svt(X, lam_s, 0.9 * thresh, max_iter=2000)
    assert np.linalg.norm(res["L"]) > 0


@pytest.fixture(scope="module")
def small_case():
    p = synth.gaussian_rpca()          # 256 x 200, rank 5, 5% outliers, k = 10
    U, V, res = _solve_factored(p, p.k)
    cvx = cv.fista_svt(p.X, p.lam_s, p.lam_l, max_iter=5000, tol=1e-13)
    return p, U, V, res, cvx


def test_factored_solve_matches_convex_solve(small_case):
    p, U, V, res, cvx = small_case
    L = U @ V.T
    relL = np.linalg.norm(L - cvx["L"]) / np.linalg.norm(cvx["L"])
    f = res["f"]
    relF = abs(f - cvx["F"]) / cvx["F"]
    print(f"L-BFGS status={res['status']} iters={res['iters']} f={f:.15g} F*={cvx['F']:.15g} "
          f"relL={relL:.2e} relF={relF:.2e} rank={cvx['rank']}")
    assert res["status"] in (lb.CONVERGED, lb.FTOL)
    assert relL <= 1e-6
    assert relF <= 1e-10


def test_solution_factors_are_balanced(small_case):
    p, U, V, res, cvx = small_case
    A, B = U.T @ U, V.T @ V
    rel = np.linalg.norm(A - B) / np.linalg.norm(A)
    # lam_l (U^T U - V^T V) is the symmetric part of U^T grad_U - V^T grad_V
    # (the G terms cancel), so the imbalance is bounded by the final gradient
    _, gU, gV = ob.objgrad(U, V, p.X, p.lam_s, p.lam_l)
    bound = (np.linalg.norm(U.T @ gU) + np.linalg.norm(V.T @ gV)) / p.lam_l
    print("balance", rel, "bound", bound / np.linalg.norm(A))
    assert np.linalg.norm(A - B) <= bound * (1 + 1e-6) + 1e-12
    assert rel <= 1e-7
    Q = np.linalg.qr(np.random.default_rng(0).normal(size=(p.k, p.k)))[0]
    f1 = ob.objective(U, V, p.X, p.lam_s, p.lam_l)
    f2 = ob.objective(U @ Q, V @ Q, p.X, p.lam_s, p.lam_l)
    assert abs(f1 - f2) <= 1e-12 * f1


def test_scipy_lbfgsb_cross_check(small_case):
    p, U, V, res, cvx = small_case
    fg = ob.make_fg(p.X, p.lam_s, p.lam_l, p.k)
    Om = synth.gaussian_matrix(p.n, p.k + 10, 11)
    U0, V0 = rs.rsvd_factors(p.X, p.k, Om)
    out = minimize(fg, ob.pack(U0, V0), jac=True, method="L-BFGS-B",
                   options=dict(maxiter=20000, ftol=1e-15, gtol=1e-11, maxcor=10))
    print("scipy f", out.fun, "oracle f", res["f"])
    assert abs(out.fun - res["f"]) <= 1e-8 * res["f"]


def test_rsvd_exact_for_low_rank_input():
    rng = np.random.default_rng(4)
    m, n, k = 120, 80, 6
    X = rng.normal(size=(m, k)) @ rng.normal(size=(k, n))
    Om = synth.gaussian_matrix(n, k + 10, 5)
    U0, V0 = rs.rsvd_factors(X, k, Om, q=0)
    assert np.linalg.norm(U0 @ V0.T - X) <= 1e-10 * np.linalg.norm(X)
    # balanced factors: U0^T U0 = V0^T V0 = Sigma
    assert np.allclose(U0.T @ U0, V0.T @ V0, atol=1e-9)


def test_rsvd_with_power_steps_matches_truncated_svd():
    rng = np.random.default_rng(5)
    m, n, k = 150, 90, 5
    s = np.concatenate([np.linspace(50, 20, k), 0.01 * np.ones(n - k)])
    Uf = np.linalg.qr(rng.normal(size=(m, n)))[0]
    Vf = np.linalg.qr(rng.normal(size=(n, n)))[0]
    X = (Uf * s) @ Vf.T
    Om = synth.gaussian_matrix(n, k + 10, 6)
    U0, V0 = rs.rsvd_factors(X, k, Om, q=2)
    best = (Uf[:, :k] * s[:k]) @ Vf[:, :k].T
    rel = np.linalg.norm(U0 @ V0.T - best) / np.linalg.norm(best)
    assert rel <= 1e-9
