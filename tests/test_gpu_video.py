"""The headline configuration against the oracle: certified solves of the
76,800 x 200 synthetic video (k = 10, rSVD start, FP32), judged by the FP64
oracle's certificate in its efficient form (Sec. 3.4: the last block's
singular values from one LAPACK SVD of the m x n projected gradient).

Bars: the oracle certifies the GPU's point (rel_gap <= 1e-3); F agrees to 1e-5;
the GPU's E and its terms agree with the oracle's within 5 % plus the floor that
FP32 evaluation of D puts on them; the leading Ritz value agrees to 1e-3."""
import numpy as np
import pytest
import torch

from oracle import certificate as ce
from paper_1702_02241_amd import rpca as R
from paper_1702_02241_amd import synth
from paper_1702_02241_amd import torch_api as T

from gpu_common import device
from test_gpu_solve import fp32_floor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def video():
    p = synth.video()
    dev = device()
    return p, T.to_device_X(p.X, dev)


@pytest.mark.parametrize("seed,precond", [(1, 1), (2, 1), (3, 0)])
def test_video_solve_certified_by_oracle(video, seed, precond):
    p, Xcm = video
    dev = device()
    ctx = T.Context(p.m, p.n, p.k, p.lam_s, p.lam_l)
    U = torch.empty(p.m, p.k, dtype=torch.float32, device=dev)
    V = torch.empty(p.n, p.k, dtype=torch.float32, device=dev)
    rc, info = ctx.solve(Xcm, U, V, init=R.RPCA_INIT_RSVD, seed=seed, certify=1, precond=precond,
                         max_iter=5000)
    torch.cuda.synchronize()
    c = ctx.certificate(Xcm, U, V)
    Ug, Vg = U.cpu().numpy().astype(np.float64), V.cpu().numpy().astype(np.float64)
    o = ce.certificate(Ug, Vg, p.X, p.lam_s, p.lam_l, tau=1e-6, form="efficient")
    e_noise, t_noise = fp32_floor(p, Ug, Vg, o["r"])
    sv0 = float(o["sv_perp"][0])
    print(f"[video seed={seed} precond={precond}] rc={rc} iters={info.iters} rounds={info.cert_rounds} "
          f"t={info.seconds * 1e3:.1f} ms | gpu F={c.F:.10g} E={c.E:.4e} rel_gap={c.rel_gap:.4e} "
          f"T=({c.T1:.3e},{c.T2:.3e},{c.T3:.3e},{c.T4:.3e}) theta0={c.theta[0]:.6f} r={c.r} | oracle "
          f"F={o['F']:.10g} E={o['E']:.4e} rel_gap={o['rel_gap']:.4e} T=({o['T1']:.3e},{o['T2']:.3e},"
          f"{o['T3']:.3e},{o['T4']:.3e}) sv0={sv0:.6f} r={o['r']} | floor E {e_noise:.2e}")
    assert rc >= 0 and info.certified == 1
    assert o["rel_gap"] <= 1e-3
    assert c.r == o["r"]
    assert abs(c.F - o["F"]) <= 1e-5 * o["F"]
    for key in ("T1", "T2", "T3"):
        assert abs(getattr(c, key) - o[key]) <= 5e-2 * o[key] + t_noise, key
    assert abs(c.E - o["E"]) <= 5e-2 * o["E"] + e_noise
    assert abs(c.theta[0] - sv0) <= 1e-3 * sv0 + 1e-6
    ctx.close()
