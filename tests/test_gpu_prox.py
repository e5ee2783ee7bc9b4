"""GPU parity of the convex baseline (accelerated proximal gradient with a
randomized singular-value threshold; the solver class of Sec. 6.1) against the
FP64 oracle's FISTA-SVT (exact LAPACK SVT).

* the first step from L = 0 is SVT_{lam_L}(-grad phi(0)) (exact SVT in the oracle),
  on instances whose threshold fits the factors;
* solves to convergence reach the convex optimum's F and rank, L matches the
  oracle's, and the certificate (Sec. 3.4) certifies the result, on shapes that
  span several tiles with ragged edges;
* a context with a mask is refused.
"""
import numpy as np
import pytest
import torch

from oracle import convex as cv
from oracle import objective as ob
from paper_1702_02241_amd import rpca as R
from paper_1702_02241_amd import synth
from paper_1702_02241_amd import torch_api as T

from gpu_common import device, f32

pytestmark = pytest.mark.gpu


def _L(U, V):
    return U.double().cpu().numpy() @ V.double().cpu().numpy().T


@pytest.mark.parametrize("m,n,lam_l", [(300, 200, 12.0), (1037, 141, 20.0)])
def test_first_step_is_the_exact_threshold(m, n, lam_l):
    # lam_L between the 4th and 5th singular values of -grad phi(0): the exact threshold has rank 4
    p = synth.gaussian_rpca(m=m, n=n, r=4, k=32, seed=500 + m, lam_s=0.3, lam_l=lam_l)
    X = f32(p.X)
    dev = device()
    ctx = T.Context(m, n, 32, p.lam_s, p.lam_l)
    rc, info, U, V = ctx.prox_solve(T.to_device_X(X, dev), max_iter=1, tol=0.0, power_steps=2)
    L1, s1 = cv.svt(-ob.grad_phi(np.zeros_like(X), X, p.lam_s), p.lam_l)
    err = np.linalg.norm(_L(U, V) - L1) / np.linalg.norm(L1)
    F1 = cv.objective(L1, X, p.lam_s, p.lam_l, sing=s1)
    print(f"[prox first step {m}x{n}] rank gpu {info.rank} oracle {s1.size}; rel L err {err:.3e}; "
          f"F {info.F:.9g} vs {F1:.9g}")
    assert info.iters == 1 and info.rank == s1.size and not info.truncated
    assert err <= 1e-4
    assert abs(info.F - F1) <= 1e-5 * F1
    ctx.close()


@pytest.mark.parametrize("m,n,r,lam_l", [(300, 200, 4, 3.0), (1037, 141, 6, 4.0), (2050, 333, 5, 6.0)])
def test_solve_reaches_the_convex_optimum_and_certifies(m, n, r, lam_l):
    p = synth.gaussian_rpca(m=m, n=n, r=r, k=32, seed=510 + m, lam_s=0.3, lam_l=lam_l)
    X = f32(p.X)
    dev = device()
    ctx = T.Context(m, n, 32, p.lam_s, p.lam_l)
    Xcm = T.to_device_X(X, dev)
    rc, info, U, V = ctx.prox_solve(Xcm, max_iter=500, tol=1e-9)
    cvx = cv.fista_svt(X, p.lam_s, p.lam_l, max_iter=20000, tol=1e-12)
    L = _L(U, V)
    err = np.linalg.norm(L - cvx["L"]) / np.linalg.norm(cvx["L"])
    cert = ctx.certificate(Xcm, U, V)
    print(f"[prox solve {m}x{n}] status {rc} iters {info.iters} restarts {info.restarts} rank {info.rank} "
          f"(oracle {cvx['rank']}) sketch {info.sketch} | F {info.F:.10g} vs F* {cvx['F']:.10g}; rel L err "
          f"{err:.3e}; certificate rel_gap {cert.rel_gap:.3e}; early steps truncated {info.truncated}; "
          f"{1000 * info.seconds:.1f} ms")
    # the first steps from L = 0 may have more values above lam_L than k (reported, not an error)
    assert rc == R.RPCA_OK
    assert info.rank == cvx["rank"]
    assert abs(info.F - cvx["F"]) <= 1e-6 * cvx["F"]
    assert err <= 1e-3
    assert cert.rel_gap <= 1e-3
    ctx.close()


def test_masked_context_is_refused():
    p = synth.partial_rpca(m=64, n=48, r=3, k=8, p_obs=0.7, seed=520)
    dev = device()
    ctx = T.Context(p.m, p.n, 8, p.lam_s, p.lam_l, mask=p.mask)
    U = torch.empty(p.m, 8, dtype=torch.float32, device=dev)
    V = torch.empty(p.n, 8, dtype=torch.float32, device=dev)
    Xcm = T.to_device_X(p.X, dev)
    assert R.rpca_prox_solve(ctx.ctx, Xcm.data_ptr(), U.data_ptr(), V.data_ptr())[0] == R.RPCA_EINVAL
    ctx.close()


def test_rank_above_the_factor_capacity_is_truncated_and_reported():
    """k = 4 factors for an optimum of rank > 4: the steps keep the top k values,
    report it, and F stays above the convex optimum."""
    p = synth.gaussian_rpca(m=120, n=80, r=6, k=4, seed=530, lam_s=0.3, lam_l=1.0)
    X = f32(p.X)
    dev = device()
    cvx = cv.fista_svt(X, p.lam_s, p.lam_l, max_iter=20000, tol=1e-12)
    ctx = T.Context(p.m, p.n, 4, p.lam_s, p.lam_l)
    rc, info, U, V = ctx.prox_solve(T.to_device_X(X, dev), max_iter=60, tol=1e-9)
    print(f"[prox truncated] status {rc} iters {info.iters} rank {info.rank} truncated {info.truncated} | F {info.F:.9g} "
          f"vs F* {cvx['F']:.9g} (rank {cvx['rank']})")
    assert cvx["rank"] > 4
    assert rc in (R.RPCA_OK, R.RPCA_ENOTCONV)
    assert info.truncated == 1 and info.rank <= 4
    assert info.F >= cvx["F"] * (1 - 1e-9)
    ctx.close()
