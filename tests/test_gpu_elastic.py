"""GPU parity of the elastic-net regulariser (r(S) = lam_s ||S||_1 + mu/2 ||S||_F^2,
marginalised like the l1 norm; Sec. 1) against the FP64 oracle.

* objective and gradient on dense, masked, ragged and multi-chunk shapes (same
  bars as the l1 objective/gradient tests); BF16 products are refused;
* mu = 0 after a nonzero mu gives results bitwise equal to a fresh l1 context;
* the certificate at an oracle optimum (terms and leading Ritz value to 1e-3);
* a certified solve whose objective matches the convex optimum of FISTA-SVT with
  the elastic marginal, and differs from the l1 optimum.
"""
import numpy as np
import pytest
import torch

from oracle import certificate as ce
from oracle import convex as cv
from oracle import lbfgs as lb
from oracle import objective as ob
from oracle import rsvd as rs
from paper_1702_02241_amd import rpca as R
from paper_1702_02241_amd import synth
from paper_1702_02241_amd import torch_api as T

from gpu_common import device, f32, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,k,p_obs,mu,prec", [
    (256, 200, 10, None, 0.2, 0),
    (37, 23, 3, None, 1.5, 0),      # ragged, m not a multiple of 4
    (1000, 300, 16, None, 0.05, 0),  # two column chunks
    (530, 129, 17, 0.5, 0.4, 0),     # masked, two rank blocks
    (4099, 513, 25, None, 0.3, 0),   # several chunks, ragged everything
])
def test_objgrad_matches_oracle(m, n, k, p_obs, mu, prec):
    if p_obs is None:
        p = synth.gaussian_rpca(m=m, n=n, r=min(5, k), k=k, seed=300 + m + n + k)
    else:
        p = synth.partial_rpca(m=m, n=n, r=min(5, k), k=k, p_obs=p_obs, seed=300 + m + n + k)
    U, V = synth.random_factors(m, n, k, 9 + k, scale=0.5)
    dev = device()
    ctx = T.Context(p.m, p.n, p.k, p.lam_s, p.lam_l, p.mask, mu=mu)
    Xcm = T.to_device_X(p.X, dev)
    f, gU, gV = ctx.objgrad(Xcm, T.to_device_factor(U, dev), T.to_device_factor(V, dev))
    fr, gUr, gVr = ob.objgrad(f32(U), f32(V), f32(p.X), p.lam_s, p.lam_l, p.mask, mu=mu)
    ef = abs(float(f.item()) - fr) / abs(fr)
    eu = rel(gU.cpu().numpy(), gUr)
    ev = rel(gV.cpu().numpy(), gVr)
    print(f"[elastic objgrad {m}x{n} k={k} mask={p_obs} mu={mu} bf16={prec}] f rel {ef:.2e} gU rel {eu:.2e} "
          f"gV rel {ev:.2e}")
    tol = 1e-5 if not prec else 1e-2
    assert ef <= (1e-5 if not prec else 1e-2)
    assert eu <= tol and ev <= tol
    ctx.close()


def test_bf16_products_are_refused_with_the_elastic_net():
    p = synth.gaussian_rpca(m=64, n=48, r=3, k=4, seed=332)
    dev = device()
    ctx = T.Context(p.m, p.n, p.k, p.lam_s, p.lam_l, mu=0.3)
    Xcm = T.to_device_X(p.X, dev)
    U, V = synth.random_factors(p.m, p.n, p.k, 3, scale=0.5)
    Ud, Vd = T.to_device_factor(U, dev), T.to_device_factor(V, dev)
    f = torch.empty(1, dtype=torch.float64, device=dev)
    gU, gV = torch.empty_like(Ud), torch.empty_like(Vd)
    rc = R.rpca_objgrad_ex(ctx.ctx, Xcm.data_ptr(), Ud.data_ptr(), Vd.data_ptr(), f.data_ptr(), gU.data_ptr(),
                           gV.data_ptr(), R.RPCA_PREC_BF16, 0)
    assert rc == R.RPCA_EINVAL
    o = R.default_opts()
    o.precision = R.RPCA_PREC_BF16_POLISH
    assert R.rpca_solve(ctx.ctx, Xcm.data_ptr(), Ud.data_ptr(), Vd.data_ptr(), o)[0] == R.RPCA_EINVAL
    ctx.close()


def test_mu_zero_is_bitwise_l1():
    p = synth.gaussian_rpca(m=530, n=129, r=5, k=17, seed=331)
    U, V = synth.random_factors(p.m, p.n, p.k, 5, scale=0.5)
    dev = device()
    Xcm = T.to_device_X(p.X, dev)
    Ud, Vd = T.to_device_factor(U, dev), T.to_device_factor(V, dev)
    a = T.Context(p.m, p.n, p.k, p.lam_s, p.lam_l)
    b = T.Context(p.m, p.n, p.k, p.lam_s, p.lam_l, mu=0.7)
    fb1, _, _ = b.objgrad(Xcm, Ud, Vd)
    b.set_elastic(0.0)
    fa, gUa, gVa = a.objgrad(Xcm, Ud, Vd)
    fb, gUb, gVb = b.objgrad(Xcm, Ud, Vd)
    assert float(fb1.item()) != float(fa.item())
    assert torch.equal(fa, fb) and torch.equal(gUa, gUb) and torch.equal(gVa, gVb)
    a.close()
    b.close()


def _instance():
    # rank(L*) = 5 with the elastic marginal (mu = 0.2); the l1 optimum has rank 3
    return synth.gaussian_rpca(m=60, n=45, r=3, k=8, seed=33, lam_s=0.3, lam_l=4.0), 0.2


def test_certificate_matches_oracle_at_an_optimum():
    p, mu = _instance()
    Om = synth.gaussian_matrix(p.n, 18, 34)
    U0, V0 = rs.rsvd_factors(p.X, 8, Om)
    res = lb.lbfgs(ob.make_fg(p.X, p.lam_s, p.lam_l, 8, mu=mu), ob.pack(U0, V0))
    U, V = ob.unpack(res["x"], p.m, p.n, 8)
    for label, (Ua, Va) in (("optimum", (U, V)), ("start", (U0, V0))):
        dev = device()
        ctx = T.Context(p.m, p.n, 8, p.lam_s, p.lam_l, mu=mu)
        c = ctx.certificate(T.to_device_X(p.X, dev), T.to_device_factor(Ua, dev), T.to_device_factor(Va, dev))
        o = ce.certificate(f32(Ua), f32(Va), f32(p.X), p.lam_s, p.lam_l, tau=1e-6, mu=mu)
        print(f"[elastic cert {label}] gpu T=({c.T1:.3e},{c.T2:.3e},{c.T3:.3e},{c.T4:.3e}) rel_gap {c.rel_gap:.3e} "
              f"| oracle T=({o['T1']:.3e},{o['T2']:.3e},{o['T3']:.3e},{o['T4']:.3e}) rel_gap {o['rel_gap']:.3e}")
        assert c.r == o["r"]
        assert abs(c.F - o["F"]) <= 1e-5 * o["F"]
        assert abs(c.phi0 - o["phi0"]) <= 1e-5 * o["phi0"]
        for key in ("T1", "T2", "T3"):
            assert abs(getattr(c, key) - o[key]) <= 1e-3 * max(o[key], 1.0) + 1e-5, key
        assert abs(c.theta[0] - o["sv_perp"][0]) <= 1e-3 * o["sv_perp"][0] + 1e-5
        if label == "optimum":
            assert c.rel_gap <= 1e-3
        ctx.close()


def test_certified_solve_reaches_the_elastic_convex_optimum():
    p, mu = _instance()
    dev = device()
    ctx = T.Context(p.m, p.n, 8, p.lam_s, p.lam_l, mu=mu)
    Xcm = T.to_device_X(p.X, dev)
    U, V = ctx.init_rsvd(Xcm)
    rc, info = ctx.solve(Xcm, U, V)
    L = U.double().cpu().numpy() @ V.double().cpu().numpy().T
    F = ob.convex_objective(L, p.X, p.lam_s, p.lam_l, mu=mu)
    cvx = cv.fista_svt(p.X, p.lam_s, p.lam_l, max_iter=20000, tol=1e-13, mu=mu)
    F_l1 = cv.fista_svt(p.X, p.lam_s, p.lam_l, max_iter=20000, tol=1e-13)["F"]
    print(f"[elastic solve] status {rc} certified {info.certified} rel_gap {info.rel_gap:.3e} iters {info.iters} "
          f"| F {F:.9g} convex F* {cvx['F']:.9g} (rank {cvx['rank']}); l1 F* {F_l1:.9g}")
    assert rc == R.RPCA_OK and info.certified
    assert F - cvx["F"] <= 1e-3 * cvx["F"]
    assert F >= cvx["F"] * (1 - 1e-6)
    assert abs(F - F_l1) > 1e-2 * cvx["F"]
    ctx.close()
