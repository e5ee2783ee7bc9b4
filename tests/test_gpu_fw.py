"""GPU parity of Frank-Wolfe with marginalisation (Sec. 6.2, Alg. 1) against
oracle.frank_wolfe.

* one iteration from an oracle iterate (L_k, t_k), on shapes that take the
  vector and scalar layouts, ragged row blocks and column chunks, the fused
  G^T G pass (n <= 256) and the separate products (n > 256), with and without
  a mask: L_{k+1}, t_{k+1} and the next iterate's F, gap and sigma;
* the start evaluated alone (max_iter = 0): F, gap, sigma, L untouched;
* a 300-iteration solve from zero: the objective never increases across calls,
  the gap bounds F - F* (FISTA-SVT), and F tracks the oracle's trajectory;
* the zero solution: lam_L above ||grad phi(0)||_2 stops at once with L = 0;
* the 76,800 x 200 video shape: one iteration from the oracle's third iterate;
* the stop test: a solve stops at the first iterate whose gap passes, unchanged;
* nonfinite input: RPCA_ENONFINITE, and the handle's next call starts cold.
"""
import numpy as np
import pytest
import torch

from oracle import convex as cv
from oracle import frank_wolfe as fw
from oracle import objective as ob
from paper_1702_02241_amd import rpca as R
from paper_1702_02241_amd import synth
from paper_1702_02241_amd import torch_api as T

from gpu_common import device, f32

pytestmark = pytest.mark.gpu

TIGHT = 3e-6  # power-iteration tolerance for parity (top Ritz pair's relative residual)


def _problem(m, n, masked, seed):
    if masked:
        return synth.partial_rpca(m=m, n=n, r=4, k=4, p_obs=0.75, seed=seed)
    return synth.gaussian_rpca(m=m, n=n, r=4, k=4, seed=seed, lam_s=0.3, lam_l=1.5)


def _to_dev(A, dev):
    """m x n host matrix -> (n, m) contiguous FP32 tensor (column-major layout)."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A, np.float32).T)).to(dev)


def _from_dev(Lcm):
    return Lcm.double().cpu().numpy().T


def _oracle_iterates(p, k):
    L, t = np.zeros((p.m, p.n)), 0.0
    for _ in range(k):
        L, t, _ = fw.fw_iteration(L, t, p.X, p.lam_s, p.lam_l, p.mask)
    return L, t


@pytest.mark.parametrize("m,n,masked", [(300, 120, False), (301, 77, True), (2084, 150, False),
                                        (2084, 150, True), (520, 300, False), (523, 301, True)])
def test_one_iteration_matches_oracle(m, n, masked):
    p = _problem(m, n, masked, 80 + m + n)
    dev = device()
    Lk, tk = _oracle_iterates(p, 4)
    Lk = f32(Lk)
    X = f32(p.X)
    solver = T.FrankWolfe(p.m, p.n, p.lam_s, p.lam_l, mask=p.mask)
    Xcm = _to_dev(X, dev)
    # the start alone
    Lcm = _to_dev(Lk, dev)
    rc0, L0, t0, info0 = solver.solve(Xcm, Lcm, tk, max_iter=0, tol=0.0, power_tol=TIGHT)
    _, _, o0 = fw.fw_iteration(Lk, tk, X, p.lam_s, p.lam_l, p.mask)
    print(f"[fw {m}x{n} mask={masked}] start: gpu F {info0.F:.9g} gap {info0.gap:.6e} sigma {info0.sigma:.8f} "
          f"power {info0.power_iters} | oracle F {o0['F']:.9g} gap {o0['gap']:.6e} sigma {o0['sigma']:.8f}")
    assert rc0 == R.RPCA_ENOTCONV and info0.iters == 0 and t0 == tk
    assert np.array_equal(_from_dev(L0), Lk)
    assert abs(info0.F - o0["F"]) <= 1e-6 * o0["F"]
    assert abs(info0.sigma - o0["sigma"]) <= 1e-5 * o0["sigma"]
    assert abs(info0.gap - o0["gap"]) <= 1e-5 * o0["F"]
    # one step
    rc, L1, t1, info = solver.solve(Xcm, _to_dev(Lk, dev), tk, max_iter=1, tol=0.0, power_tol=TIGHT)
    L1o, t1o, step_o = fw.fw_iteration(Lk, tk, X, p.lam_s, p.lam_l, p.mask)
    _, _, o1 = fw.fw_iteration(L1o, t1o, X, p.lam_s, p.lam_l, p.mask)
    Lg = _from_dev(L1)
    err = np.linalg.norm(Lg - L1o) / np.linalg.norm(L1o)
    print(f"  step: eta gpu {info.eta:.8f} oracle {step_o['eta']:.8f}; t {t1:.9g} vs {t1o:.9g}; "
          f"||L - L_oracle|| / ||L_oracle|| {err:.3e}; F {info.F:.9g} vs {o1['F']:.9g}; "
          f"gap {info.gap:.6e} vs {o1['gap']:.6e}")
    assert info.iters == 1
    assert abs(info.eta - step_o["eta"]) <= 1e-4 * max(step_o["eta"], 1e-3)
    assert abs(t1 - t1o) <= 1e-5 * t1o
    assert err <= 1e-4
    assert abs(info.F - o1["F"]) <= 1e-5 * o1["F"]
    assert abs(info.sigma - o1["sigma"]) <= 1e-4 * o1["sigma"]
    assert abs(info.gap - o1["gap"]) <= 1e-4 * o1["F"]
    solver.close()


@pytest.mark.parametrize("masked", [False, True])
def test_solve_from_zero_tracks_oracle_and_gap_bounds_suboptimality(masked):
    p = _problem(120, 90, masked, 90 + masked)
    dev = device()
    F_star = cv.fista_svt(p.X, p.lam_s, p.lam_l, mask=p.mask, max_iter=20000, tol=1e-13)["F"]
    solver = T.FrankWolfe(p.m, p.n, p.lam_s, p.lam_l, mask=p.mask)
    Xcm = _to_dev(p.X, dev)
    Lcm, t, F_prev = None, 0.0, np.inf
    for chunk in range(6):
        rc, Lcm, t, info = solver.solve(Xcm, Lcm, t, max_iter=50, tol=0.0)
        assert info.F <= F_prev * (1 + 1e-6)
        assert info.F - F_star <= info.gap * (1 + 1e-3) + 1e-5 * F_star
        F_prev = info.F
    res = fw.fw_solve(p.X, p.lam_s, p.lam_l, p.mask, max_iter=300, tol=0.0)
    L = _from_dev(Lcm)
    s = np.linalg.svd(L, compute_uv=False)
    print(f"[fw solve mask={masked}] 300 iterations: gpu F {info.F:.9g} gap {info.gap:.4e} | oracle F "
          f"{res['F']:.9g} gap {res['gap']:.4e} | F* {F_star:.9g}; ||L||_* {s.sum():.6g} t {t:.6g}")
    assert abs(info.F - res["F"]) <= 2e-3 * res["F"]
    assert s.sum() <= t * (1 + 1e-4)
    assert abs(ob.phi(L, p.X, p.lam_s, p.mask) + p.lam_l * t - info.F) <= 1e-5 * info.F
    solver.close()


def test_zero_solution_stops_at_once():
    p = synth.gaussian_rpca(m=64, n=40, r=2, k=2, seed=95, lam_s=0.5, lam_l=1.0)
    g0 = np.linalg.norm(ob.grad_phi(np.zeros_like(p.X), p.X, p.lam_s), 2)
    dev = device()
    solver = T.FrankWolfe(p.m, p.n, p.lam_s, 1.01 * g0)
    rc, Lcm, t, info = solver.solve(_to_dev(p.X, dev), None, 0.0, max_iter=10, tol=1e-9)
    assert rc == R.RPCA_OK and info.iters == 0 and not info.last_step
    assert info.gap == 0.0 and t == 0.0 and float(Lcm.abs().max()) == 0.0
    solver.close()


def test_video_shape_one_iteration_matches_oracle():
    """76,800 x 200 (the synthetic video workload): one GPU iteration from the
    oracle's third iterate against the oracle's fourth."""
    v = synth.video()
    X = f32(v.X)
    m, n = X.shape
    lam_s, lam_l = v.lam_s, v.lam_l
    L, t = np.zeros((m, n)), 0.0
    for _ in range(3):
        L, t, _ = fw.fw_iteration(L, t, X, lam_s, lam_l)
    L = f32(L)
    L4, t4, st = fw.fw_iteration(L, t, X, lam_s, lam_l)
    dev = device()
    solver = T.FrankWolfe(m, n, lam_s, lam_l)
    rc, Lg, tg, info = solver.solve(_to_dev(X, dev), _to_dev(L, dev), t, max_iter=1, tol=0.0, power_tol=TIGHT)
    err = np.linalg.norm(_from_dev(Lg) - L4) / np.linalg.norm(L4)
    print(f"[fw video {m}x{n}] eta {info.eta:.8f} vs {st['eta']:.8f}; t {tg:.9g} vs {t4:.9g}; rel L err {err:.3e}; "
          f"power steps {info.power_iters}")
    assert abs(tg - t4) <= 1e-5 * t4
    assert err <= 1e-4
    solver.close()


@pytest.mark.parametrize("m,n,masked", [(90, 5, False), (64, 3, True), (37, 1, False)])
def test_fewer_columns_than_the_power_block(m, n, masked):
    """n < 8: the power block shrinks to n columns (zero padding in the kernels);
    one iteration from the oracle's second iterate against the oracle's third."""
    if masked:
        p = synth.partial_rpca(m=m, n=n, r=1, k=1, p_obs=0.8, seed=97 + n)
    else:
        p = synth.gaussian_rpca(m=m, n=n, r=1, k=1, seed=97 + n, lam_s=0.3, lam_l=0.5)
    dev = device()
    X = f32(p.X)
    L, t = np.zeros((m, n)), 0.0
    for _ in range(2):
        L, t, _ = fw.fw_iteration(L, t, X, p.lam_s, p.lam_l, p.mask)
    L = f32(L)
    L3, t3, st = fw.fw_iteration(L, t, X, p.lam_s, p.lam_l, p.mask)
    solver = T.FrankWolfe(m, n, p.lam_s, p.lam_l, mask=p.mask)
    rc, Lg, tg, info = solver.solve(_to_dev(X, dev), _to_dev(L, dev), t, max_iter=1, tol=0.0, power_tol=TIGHT)
    Lgh = _from_dev(Lg)
    den = max(np.linalg.norm(L3), 1e-30)
    err = np.linalg.norm(Lgh - L3) / den
    print(f"[fw small n {m}x{n} mask={masked}] sigma step {st['sigma']:.6f} eta {info.eta:.8f} vs {st['eta']:.8f}; "
          f"t {tg:.9g} vs {t3:.9g}; rel L err {err:.3e}")
    assert abs(tg - t3) <= 1e-5 * max(t3, 1e-12) + 1e-12
    assert err <= 1e-4
    solver.close()


@pytest.mark.parametrize("m,n,masked", [(300, 120, False), (301, 77, True), (520, 300, False)])
def test_stops_at_the_gap_test_with_that_iterate(m, n, masked):
    """The stop test on the device (gap <= tol F, Alg. 1): with tol just above the
    gap ratio of iterate 25, a solve from zero stops at the first iterate j <= 25
    that passes, returns that iterate unchanged (bitwise the one max_iter = j
    returns with tol = 0), and iterate j - 1 does not pass.  Fresh handles for
    each solve, so every one starts from the same power block."""
    p = _problem(m, n, masked, seed=41 + n)
    dev = device()
    Xcm = _to_dev(p.X, dev)

    def run(max_iter, tol):
        solver = T.FrankWolfe(m, n, p.lam_s, p.lam_l, mask=p.mask)
        out = solver.solve(Xcm, None, 0.0, max_iter=max_iter, tol=tol)
        solver.close()
        return out

    rc, _, _, info = run(25, 0.0)
    assert rc == R.RPCA_ENOTCONV and info.iters == 25
    tol = info.gap / info.F * (1 + 1e-9)
    rc, Lj, tj, infoj = run(1000, tol)
    j = infoj.iters
    print(f"[fw stop {m}x{n} mask={masked}] tol {tol:.6e}: stopped at {j}, gap/F {infoj.gap / infoj.F:.6e}")
    assert rc == R.RPCA_OK and 0 < j <= 25
    assert infoj.gap <= tol * infoj.F
    rc0, L0, t0, info0 = run(j, 0.0)
    assert rc0 == R.RPCA_ENOTCONV and info0.iters == j
    assert info0.F == infoj.F and info0.gap == infoj.gap and t0 == tj
    assert torch.equal(L0, Lj)
    rcp, _, _, infop = run(j - 1, tol)
    assert rcp == R.RPCA_ENOTCONV and infop.iters == j - 1
    assert infop.gap > tol * infop.F


@pytest.mark.parametrize("where", ["X", "L"])
def test_nonfinite_input_reports_and_the_next_call_starts_clean(where):
    """An observed NaN in X (or Inf in the start L) makes phi nonfinite: the solve
    returns RPCA_ENONFINITE, and a later solve on clean data with the same handle
    is bitwise that of a fresh handle (the power block is not reused)."""
    p = _problem(300, 120, False, seed=43)
    dev = device()
    Xcm = _to_dev(p.X, dev)
    Lbad = torch.zeros_like(Xcm)
    Xbad = Xcm.clone()
    if where == "X":
        Xbad[7, 5] = float("nan")
    else:
        Lbad[7, 5] = float("inf")
    solver = T.FrankWolfe(p.m, p.n, p.lam_s, p.lam_l)
    rc, t, _ = R.rpca_fw_solve(solver.h, Xbad.data_ptr(), Lbad.data_ptr(), 0.0, 10, 0.0, 0.0, T._stream())
    torch.cuda.synchronize()
    assert rc == R.RPCA_ENONFINITE
    rc1, L1, t1, info1 = solver.solve(Xcm, None, 0.0, max_iter=10, tol=0.0)
    solver.close()
    fresh = T.FrankWolfe(p.m, p.n, p.lam_s, p.lam_l)
    rc2, L2, t2, info2 = fresh.solve(Xcm, None, 0.0, max_iter=10, tol=0.0)
    fresh.close()
    print(f"[fw nonfinite {where}] then F {info1.F:.9g} vs fresh {info2.F:.9g}")
    assert rc1 == rc2 == R.RPCA_ENOTCONV and info1.iters == info2.iters == 10
    assert info1.F == info2.F and t1 == t2 and torch.equal(L1, L2)
