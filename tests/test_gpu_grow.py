"""GPU parity of rank growth (Sec. 4.1, read with the certificate's last block)
against oracle.rank_growth and the convex solver oracle.convex.

* rpca_rank_direction at a stationary point of a too-small rank bound: sigma
  to 1e-3 of the oracle's exact top singular value of P_U^perp D P_V^perp; the
  GPU pair is orthogonal to L's column and row spaces, has u^T D v = sigma (D in
  FP64 by the oracle), and the grown factors lower f by the guaranteed bound;
* at a certified optimum: sigma <= 1 and a zero column pair;
* rpca_solve_grow from a rank below rank(L*): the solve certifies and its F is
  within the certified gap of the convex optimum (FISTA-SVT), dense and masked.
"""
import numpy as np
import pytest
import torch

from oracle import certificate as ce
from oracle import convex as cv
from oracle import lbfgs as lb
from oracle import objective as ob
from oracle import rank_growth as rg
from oracle import rsvd as rs
from paper_1702_02241_amd import rpca as R
from paper_1702_02241_amd import synth
from paper_1702_02241_amd import torch_api as T

from gpu_common import device, f32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stationary():
    """80 x 60, rank(L*) = 6, stationary point of the k = 3 factorisation (oracle L-BFGS)."""
    p = synth.gaussian_rpca(m=80, n=60, r=6, k=3, seed=27, lam_s=0.2, lam_l=2.0)
    Om = synth.gaussian_matrix(p.n, 13, 28)
    U0, V0 = rs.rsvd_factors(p.X, 3, Om)
    res = lb.lbfgs(ob.make_fg(p.X, p.lam_s, p.lam_l, 3), ob.pack(U0, V0))
    U, V = ob.unpack(res["x"], p.m, p.n, 3)
    return p, f32(U), f32(V)


def test_rank_direction_matches_oracle(stationary):
    p, U, V = stationary
    dev = device()
    ctx = T.Context(p.m, p.n, 3, p.lam_s, p.lam_l)
    Xcm = T.to_device_X(p.X, dev)
    sigma, t, uc, vc = ctx.rank_direction(Xcm, T.to_device_factor(U, dev), T.to_device_factor(V, dev))
    ctx.close()
    X = f32(p.X)
    s_o, u_o, v_o = rg.growth_direction(U, V, X, p.lam_s, p.lam_l)
    print(f"[grow 80x60 k=3] gpu sigma {sigma:.8f} t {t:.6e} | oracle sigma {s_o:.8f}")
    assert s_o > 1.01
    assert abs(sigma - s_o) <= 1e-3 * s_o
    assert abs(t - p.lam_l * (sigma - 1.0)) <= 1e-12 * max(t, 1.0)
    u = uc.double().cpu().numpy() / np.sqrt(t)
    v = -vc.double().cpu().numpy() / np.sqrt(t)
    assert abs(np.linalg.norm(u) - 1) <= 1e-5 and abs(np.linalg.norm(v) - 1) <= 1e-5
    # orthogonal to L's column and row spaces
    U1, _, V1, _ = ce.factor_svd(U, V, 1e-10)
    assert np.linalg.norm(U1.T @ u) <= 1e-4
    assert np.linalg.norm(V1.T @ v) <= 1e-4
    # the pair attains the top singular value of the projected block
    D = ob.grad_phi(U @ V.T, X, p.lam_s) / p.lam_l
    assert abs(u @ D @ v - s_o) <= 1e-3 * s_o
    # the rank-one update agrees with the oracle's (sign-free)
    assert np.linalg.norm(np.outer(u, v) - np.outer(u_o, v_o)) <= 2e-2
    # appending the FP32 columns lowers f by the guaranteed bound (less a rounding margin)
    Ug = np.concatenate([U, f32(uc.cpu().numpy())[:, None]], axis=1)
    Vg = np.concatenate([V, f32(vc.cpu().numpy())[:, None]], axis=1)
    f0 = ob.objective(U, V, X, p.lam_s, p.lam_l)
    f1 = ob.objective(Ug, Vg, X, p.lam_s, p.lam_l)
    bound = rg.decrease_bound(s_o, p.lam_l)
    print(f"  f {f0:.8g} -> {f1:.8g}: decrease {f0 - f1:.6e}, bound {bound:.6e}")
    assert f0 - f1 >= bound * (1 - 1e-2)
    # the GPU objective at the grown factors agrees
    ctx4 = T.Context(p.m, p.n, 4, p.lam_s, p.lam_l)
    fg, _, _ = ctx4.objgrad(Xcm, T.to_device_factor(Ug, dev), T.to_device_factor(Vg, dev))
    ctx4.close()
    assert abs(float(fg.item()) - f1) <= 1e-5 * abs(f1)


def test_rank_direction_is_zero_at_a_certified_optimum():
    p = synth.gaussian_rpca(m=150, n=100, r=4, k=6, seed=43, lam_s=0.2, lam_l=2.0)   # rank(L*) = 4
    dev = device()
    ctx = T.Context(p.m, p.n, 6, p.lam_s, p.lam_l)
    Xcm = T.to_device_X(p.X, dev)
    U, V = ctx.init_rsvd(Xcm)
    rc, info = ctx.solve(Xcm, U, V)
    assert rc == R.RPCA_OK and info.certified
    sigma, t, uc, vc = ctx.rank_direction(Xcm, U, V)
    ctx.close()
    print(f"[grow at optimum] sigma {sigma:.6f} rel_gap {info.rel_gap:.3e}")
    assert sigma <= 1.0 + 1e-3
    if sigma <= 1.0:
        assert t == 0.0
        assert float(uc.abs().max()) == 0.0 and float(vc.abs().max()) == 0.0


@pytest.mark.parametrize("case", ["dense 80x60 rank 6 from k0=3", "masked 120x90 rank 5 from k0=2"])
def test_solve_grow_certifies_from_too_small_rank(case):
    if case.startswith("dense"):
        p = synth.gaussian_rpca(m=80, n=60, r=6, k=3, seed=27, lam_s=0.2, lam_l=2.0)
        k0, k_max = 3, 10
    else:
        p = synth.partial_rpca(m=120, n=90, r=5, k=2, p_obs=0.7, seed=41)
        k0, k_max = 2, 10
    dev = device()
    Xcm = T.to_device_X(p.X, dev)
    rc, info, U, V = T.solve_grow(Xcm, p.m, p.n, k0, k_max, p.lam_s, p.lam_l, mask=p.mask)
    k = U.shape[1]
    Ug = U.double().cpu().numpy()
    Vg = V.double().cpu().numpy()
    cvx = cv.fista_svt(p.X, p.lam_s, p.lam_l, mask=p.mask, max_iter=20000, tol=1e-12)
    L = Ug @ Vg.T
    F = ob.phi(L, p.X, p.lam_s, p.mask) + p.lam_l * np.sum(np.linalg.svd(L, compute_uv=False))
    print(f"[solve_grow {case}] status {rc} k {k0}->{k} certified {info.certified} "
          f"rel_gap {info.rel_gap:.3e} iters {info.iters} cert_rounds {info.cert_rounds} | "
          f"F {F:.9g} convex F {cvx['F']:.9g} rank(L*) {cvx['rank']}")
    assert rc == R.RPCA_OK and info.certified
    assert cvx["rank"] <= k <= k_max and k > k0
    assert F - cvx["F"] <= 1e-3 * cvx["F"]
    assert F >= cvx["F"] * (1 - 1e-6)
