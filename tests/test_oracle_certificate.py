"""Pins for oracle.certificate (Sec. 3.4).

* the exact form (complete bases, four blocks) and the efficient form
  (cheap identities + SVD of the projected gradient) agree;
* ~0 at the convex optimum computed by the independent FISTA-SVT solver;
* the gap bound dominates the true suboptimality F(L_t) - F* along iterates;
* at U = V = 0 the certificate equals sum (sigma_i(D) - 1)_+^2 from LAPACK;
* it plateaus away from zero when k < rank(L*) (the behaviour of Fig. CertTests);
* the factor-based SVD (footnote) reproduces LAPACK's SVD of U V^T.
"""
import numpy as np

from oracle import certificate as ce
from oracle import convex as cv
from oracle import lbfgs as lb
from oracle import objective as ob
from oracle import rsvd as rs
from paper_1702_02241_amd import synth


def test_factor_svd_matches_lapack():
    rng = np.random.default_rng(0)
    U, V = rng.normal(size=(50, 6)), rng.normal(size=(40, 6))
    U1, sig, V1, _ = ce.factor_svd(U, V)
    s = np.linalg.svd(U @ V.T, compute_uv=False)
    assert np.allclose(sig, s[:6], rtol=1e-12)
    assert np.allclose((U1 * sig) @ V1.T, U @ V.T, atol=1e-10)
    assert np.allclose(U1.T @ U1, np.eye(6), atol=1e-12)


def test_exact_and_efficient_forms_agree_off_optimum():
    p = synth.gaussian_rpca(m=60, n=45, r=3, k=6, seed=21)
    U, V = synth.random_factors(p.m, p.n, p.k, 22, scale=0.5)
    a = ce.certificate(U, V, p.X, p.lam_s, p.lam_l, form="exact")
    b = ce.certificate(U, V, p.X, p.lam_s, p.lam_l, form="efficient")
    for key in ("T1", "T2", "T3", "T4", "E", "gap"):
        print(key, a[key], b[key])
        assert abs(a[key] - b[key]) <= 1e-10 * max(1.0, abs(a[key]))
    assert abs(a["normM2"] - b["normM2"]) <= 1e-9 * max(1.0, a["normM2"])


def test_zero_factors_reduce_to_spectral_formula():
    p = synth.gaussian_rpca(m=40, n=30, r=3, k=4, seed=23, lam_l=0.05)
    U, V = np.zeros((p.m, p.k)), np.zeros((p.n, p.k))
    c = ce.certificate(U, V, p.X, p.lam_s, p.lam_l)
    D = ob.grad_phi(np.zeros_like(p.X), p.X, p.lam_s) / p.lam_l
    sv = np.linalg.svd(D, compute_uv=False)
    expect = float(np.sum(np.maximum(sv - 1, 0) ** 2))
    assert c["r"] == 0 and c["T1"] == 0 and c["T2"] == 0 and c["T3"] == 0
    assert abs(c["T4"] - expect) <= 1e-12 * max(1, expect)


def test_certificate_vanishes_at_convex_optimum():
    p = synth.gaussian_rpca(m=80, n=60, r=3, k=8, seed=24, lam_s=0.15)
    cvx = cv.fista_svt(p.X, p.lam_s, p.lam_l, max_iter=20000, tol=1e-14)
    Uf, s, Vt = np.linalg.svd(cvx["L"], full_matrices=False)
    r = cvx["rank"]
    U = Uf[:, :r] * np.sqrt(s[:r])
    V = Vt[:r].T * np.sqrt(s[:r])
    c = ce.certificate(U, V, p.X, p.lam_s, p.lam_l)
    print("cert at convex optimum", c["E"], c["rel_gap"], "iters", cvx["iters"])
    assert c["E"] <= 1e-6
    assert c["rel_gap"] <= 1e-7


def test_gap_bound_dominates_true_gap_along_iterates():
    p = synth.gaussian_rpca(m=80, n=60, r=3, k=8, seed=25, lam_s=0.15)
    F_star = cv.fista_svt(p.X, p.lam_s, p.lam_l, max_iter=20000, tol=1e-14)["F"]
    U0, V0 = synth.random_factors(p.m, p.n, p.k, 26, scale=0.3)
    seen = []

    def cb(it, x, f, g):
        if it % 5 == 0:
            U, V = ob.unpack(x, p.m, p.n, p.k)
            seen.append(ce.certificate(U, V, p.X, p.lam_s, p.lam_l, tau=1e-12))

    lb.lbfgs(ob.make_fg(p.X, p.lam_s, p.lam_l, p.k), ob.pack(U0, V0), max_iter=200, callback=cb)
    assert len(seen) >= 10
    for c in seen:
        true_gap = c["F"] - F_star
        assert c["gap"] >= true_gap - 1e-9 * F_star


def test_certificate_plateaus_when_rank_bound_too_small():
    p = synth.gaussian_rpca(m=80, n=60, r=6, k=3, seed=27, lam_s=0.2, lam_l=0.5)
    cvx = cv.fista_svt(p.X, p.lam_s, p.lam_l, max_iter=20000, tol=1e-13)
    assert cvx["rank"] > 3
    Om = synth.gaussian_matrix(p.n, 13, 28)
    U0, V0 = rs.rsvd_factors(p.X, 3, Om)
    res = lb.lbfgs(ob.make_fg(p.X, p.lam_s, p.lam_l, 3), ob.pack(U0, V0))
    U, V = ob.unpack(res["x"], p.m, p.n, 3)
    c = ce.certificate(U, V, p.X, p.lam_s, p.lam_l)
    print("plateau T4", c["T4"], "rel_gap", c["rel_gap"], "true rank", cvx["rank"])
    # stationary for the factored problem (T1..T3 ~ 0) but not optimal: T4 stays positive
    assert c["T1"] + c["T2"] + c["T3"] <= 1e-10
    assert c["T4"] > 1e-3
    assert not c["certified"]
