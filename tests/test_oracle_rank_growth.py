"""Pins for oracle.rank_growth (Sec. 4.1, read with the certificate's last block).

* the grown factors lower f by at least lam_l^2 (sigma - 1)^2 / 2, at random
  points and at a stationary point of a too-small rank bound;
* the derivative of f along the balanced pair (sqrt(t) u, -sqrt(t) v) at t = 0+
  is lam_l (1 - sigma), by a one-sided second-order difference in t (f as a
  function of t is phi(L - t u v^T) + lam_l/2 (||U||^2 + ||V||^2) + lam_l t);
* sigma is the top singular value of the certificate's projected block: the
  certificate's T4 includes (sigma - 1)_+^2;
* sigma <= 1 at the convex optimum (FISTA-SVT, an independent solver), and > 1
  at a stationary point with k < rank(L*); growing there and re-solving reaches
  the convex optimum's objective.
"""
import numpy as np

from oracle import certificate as ce
from oracle import convex as cv
from oracle import lbfgs as lb
from oracle import objective as ob
from oracle import rank_growth as rg
from oracle import rsvd as rs
from paper_1702_02241_amd import synth


def _stationary_low_rank():
    p = synth.gaussian_rpca(m=80, n=60, r=6, k=3, seed=27, lam_s=0.2, lam_l=2.0)  # rank(L*) = 6
    Om = synth.gaussian_matrix(p.n, 13, 28)
    U0, V0 = rs.rsvd_factors(p.X, 3, Om)
    res = lb.lbfgs(ob.make_fg(p.X, p.lam_s, p.lam_l, 3), ob.pack(U0, V0))
    U, V = ob.unpack(res["x"], p.m, p.n, 3)
    return p, U, V


def test_growth_decreases_f_by_the_bound():
    p, U, V = _stationary_low_rank()
    cases = [("stationary k=3", U, V)]
    for seed in (31, 32):
        Ur, Vr = synth.random_factors(p.m, p.n, 3, seed, scale=0.3)
        cases.append((f"random {seed}", Ur, Vr))
    grew = 0
    for label, Ua, Va in cases:
        f0 = ob.objective(Ua, Va, p.X, p.lam_s, p.lam_l)
        Un, Vn, sigma, t = rg.grow(Ua, Va, p.X, p.lam_s, p.lam_l)
        f1 = ob.objective(Un, Vn, p.X, p.lam_s, p.lam_l)
        bound = rg.decrease_bound(sigma, p.lam_l)
        print(f"{label}: sigma {sigma:.6f} t {t:.4e} f {f0:.8g} -> {f1:.8g} (decrease {f0 - f1:.4e}, bound {bound:.4e})")
        if sigma > 1:
            grew += 1
            assert Un.shape[1] == Ua.shape[1] + 1
            assert f0 - f1 >= bound * (1 - 1e-9)
        else:
            assert f1 == f0
    assert grew >= 1


def test_directional_derivative_is_lam_l_times_one_minus_sigma():
    p, U, V = _stationary_low_rank()
    sigma, u, v = rg.growth_direction(U, V, p.X, p.lam_s, p.lam_l)
    L = U @ V.T

    def f_of_t(t):  # f at the grown factors [U, sqrt(t) u], [V, -sqrt(t) v]
        return ob.phi(L - t * np.outer(u, v), p.X, p.lam_s) + 0.5 * p.lam_l * (
            np.sum(U * U) + np.sum(V * V) + 2 * t)

    # one-sided (t >= 0), second order: exact for the piecewise-quadratic f(t) when no
    # entry changes Huber branch within [0, 2h]
    h = 1e-6
    d_num = (-3 * f_of_t(0.0) + 4 * f_of_t(h) - f_of_t(2 * h)) / (2 * h)
    print("sigma", sigma, "numeric", d_num, "predicted", p.lam_l * (1 - sigma))
    assert abs(d_num - p.lam_l * (1 - sigma)) <= 1e-5 * max(1.0, abs(p.lam_l * (1 - sigma)))


def test_sigma_is_the_certificate_last_block():
    p, U, V = _stationary_low_rank()
    sigma, _, _ = rg.growth_direction(U, V, p.X, p.lam_s, p.lam_l)
    c = ce.certificate(U, V, p.X, p.lam_s, p.lam_l)
    print("sigma", sigma, "sv_perp[0]", c["sv_perp"][0], "T4", c["T4"])
    assert abs(sigma - c["sv_perp"][0]) <= 1e-10 * max(1.0, sigma)
    assert c["T4"] >= (sigma - 1) ** 2 * (1 - 1e-12)


def test_sigma_below_one_at_optimum_and_growth_reaches_it():
    p, U, V = _stationary_low_rank()
    cvx = cv.fista_svt(p.X, p.lam_s, p.lam_l, max_iter=20000, tol=1e-13)
    assert cvx["rank"] > 3
    Uf, s, Vt = np.linalg.svd(cvx["L"], full_matrices=False)
    r = cvx["rank"]
    sig_opt, _, _ = rg.growth_direction(Uf[:, :r] * np.sqrt(s[:r]), Vt[:r].T * np.sqrt(s[:r]), p.X,
                                        p.lam_s, p.lam_l)
    sig_k3, _, _ = rg.growth_direction(U, V, p.X, p.lam_s, p.lam_l)
    print("sigma at the convex optimum", sig_opt, "at the k=3 stationary point", sig_k3)
    assert sig_opt <= 1 + 1e-6
    assert sig_k3 > 1.01
    # grow and re-solve until sigma <= 1: the objective reaches the convex optimum's
    Ug, Vg = U, V
    for _ in range(8):
        Ug, Vg, sig, t = rg.grow(Ug, Vg, p.X, p.lam_s, p.lam_l)
        if t == 0:
            break
        kk = Ug.shape[1]
        res = lb.lbfgs(ob.make_fg(p.X, p.lam_s, p.lam_l, kk), ob.pack(Ug, Vg))
        Ug, Vg = ob.unpack(res["x"], p.m, p.n, kk)
    F_grown = ob.objective(Ug, Vg, p.X, p.lam_s, p.lam_l)
    s_g = np.linalg.svd(Ug @ Vg.T, compute_uv=False)
    F_conv = ob.phi(Ug @ Vg.T, p.X, p.lam_s) + p.lam_l * np.sum(s_g)
    print("grown to k", Ug.shape[1], "F", F_conv, "convex optimum F", cvx["F"])
    assert abs(F_conv - cvx["F"]) <= 1e-6 * cvx["F"]
    assert F_grown >= F_conv - 1e-9 * abs(F_conv)
