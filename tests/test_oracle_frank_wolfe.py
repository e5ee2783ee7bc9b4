"""Pins for oracle.frank_wolfe (Sec. 6.2, Alg. 1 with the readings in its header).

* the closed-form step size minimises the quadratic model (brute force on a grid
  refined by golden section), dense and masked;
* at every iterate the Frank-Wolfe gap bounds F_k - F*, with F* from FISTA-SVT
  (oracle.convex, an independent solver); F_k never increases; ||L_k||_* <= t_k;
* lam_s -> infinity with every entry observed: phi = 1/2||L - X||^2 and the
  optimum is the singular-value soft threshold of X; F - F* >= 1/2||L - L*||^2
  (strong convexity) ties the iterate to it;
* lam_l >= ||grad phi(0)||_2: the first vertex is 0 and the solve stops at L = 0.
"""
import numpy as np
import pytest

from oracle import convex as cv
from oracle import frank_wolfe as fw
from oracle import objective as ob
from paper_1702_02241_amd import synth


def _model(G, L, t, V, Vt, lam_l, W, eta):
    D = W * (V - L)
    R = G + eta * D
    return 0.5 * float(np.sum(R * R)) + lam_l * ((1 - eta) * t + eta * Vt)


@pytest.mark.parametrize("masked", [False, True])
def test_step_size_minimises_the_model(masked):
    rng = np.random.default_rng(5 + masked)
    for trial in range(6):
        m, n = 12, 9
        G = rng.normal(size=(m, n))
        L = rng.normal(size=(m, n))
        V = rng.normal(size=(m, n)) * (0.1 if trial % 2 else 3.0)
        t, Vt = abs(rng.normal()) * 3, abs(rng.normal()) * 3
        lam_l = abs(rng.normal()) + 0.1
        mask = (rng.random((m, n)) < 0.7).astype(np.uint8) if masked else None
        W = np.ones((m, n)) if mask is None else mask.astype(np.float64)
        if masked:
            G = G * W
        eta = fw.step_size(G, L, t, V, Vt, lam_l, mask)
        grid = np.linspace(0.0, 1.0, 20001)
        vals = [_model(G, L, t, V, Vt, lam_l, W, e) for e in grid]
        best = grid[int(np.argmin(vals))]
        lo, hi = max(0.0, best - 1e-4), min(1.0, best + 1e-4)
        gr = (np.sqrt(5) - 1) / 2
        for _ in range(80):
            a = hi - gr * (hi - lo)
            b = lo + gr * (hi - lo)
            if _model(G, L, t, V, Vt, lam_l, W, a) < _model(G, L, t, V, Vt, lam_l, W, b):
                hi = b
            else:
                lo = a
        brute = 0.5 * (lo + hi)
        assert abs(eta - brute) <= 1e-7, (trial, eta, brute)


@pytest.mark.parametrize("masked", [False, True])
def test_gap_bounds_suboptimality_and_objective_never_increases(masked):
    if masked:
        p = synth.partial_rpca(m=40, n=30, r=3, k=3, p_obs=0.7, seed=71)
    else:
        p = synth.gaussian_rpca(m=40, n=30, r=3, k=3, seed=70, lam_s=0.3, lam_l=1.0)
    F_star = cv.fista_svt(p.X, p.lam_s, p.lam_l, mask=p.mask, max_iter=20000, tol=1e-13)["F"]
    L, t = np.zeros_like(p.X), 0.0
    F_prev = np.inf
    for it in range(400):
        Ln, tn, info = fw.fw_iteration(L, t, p.X, p.lam_s, p.lam_l, p.mask)
        assert info["F"] - F_star <= info["gap"] * (1 + 1e-9) + 1e-9 * F_star, (it, info)
        assert info["F"] <= F_prev * (1 + 1e-12), it
        assert np.sum(np.linalg.svd(L, compute_uv=False)) <= t * (1 + 1e-9) + 1e-12, it
        F_prev = info["F"]
        L, t = Ln, tn
    print("masked" if masked else "dense", "after 400 iterations: F", info["F"], "F*", F_star, "gap", info["gap"])
    assert info["F"] - F_star <= 2e-2 * F_star


def test_converges_to_the_svt_closed_form():
    rng = np.random.default_rng(9)
    m, n, lam_l = 30, 20, 2.0
    X = rng.normal(size=(m, 3)) @ rng.normal(size=(3, n)) + 0.3 * rng.normal(size=(m, n))
    lam_s = 1e6  # every residual stays on the quadratic branch
    L_star, s_star = cv.svt(X, lam_l)
    F_star = lam_l * float(np.sum(s_star)) + 0.5 * float(np.sum((L_star - X) ** 2))
    res = fw.fw_solve(X, lam_s, lam_l, max_iter=5000, tol=1e-6)
    F = res["F"]
    dist2 = float(np.sum((res["L"] - L_star) ** 2))
    print("iters", res["iters"], "F", F, "F*", F_star, "gap", res["gap"], "||L - L*||^2", dist2)
    assert F - F_star <= res["gap"] + 1e-9 * F_star
    assert F - F_star <= 1e-5 * F_star
    # lam_l t + phi(L) >= F(L) >= F* + 1/2||L - L*||^2
    assert 0.5 * dist2 <= F - F_star + 1e-9 * F_star


def test_zero_solution_when_lam_l_exceeds_the_gradient_norm():
    p = synth.gaussian_rpca(m=30, n=25, r=2, k=2, seed=72, lam_s=0.5, lam_l=1.0)
    g0 = np.linalg.norm(ob.grad_phi(np.zeros_like(p.X), p.X, p.lam_s), 2)
    res = fw.fw_solve(p.X, p.lam_s, 1.01 * g0, max_iter=10, tol=1e-12)
    assert res["iters"] == 0 and not res["hist"][0]["step"]
    assert res["gap"] == 0.0 and float(np.abs(res["L"]).max()) == 0.0
