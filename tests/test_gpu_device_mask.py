"""Contexts made from a device bitmask (rpca_create_device_mask) against contexts
made from the host mask: the same packed mask, so the objective/gradient and a
certified solve are bitwise the same; and both at oracle parity.  Bits past row
m - 1 of the device mask (set on purpose here) are cleared by the copy."""
import numpy as np
import pytest
import torch

from oracle import objective as ob
from paper_1702_02241_amd import rpca as R
from paper_1702_02241_amd import synth
from paper_1702_02241_amd import torch_api as T

from gpu_common import device, f32, rel

pytestmark = pytest.mark.gpu


def _pack_mask_dirty(mask):
    """Column-major device bitmask (bit i % 32 of word j*ceil(m/32) + i/32), with the
    bits past row m - 1 set."""
    m, n = mask.shape
    mw = (m + 31) // 32
    cols = np.ones((n, mw * 32), np.uint8)
    cols[:, :m] = (np.asarray(mask) != 0).T
    words = np.packbits(cols, axis=1, bitorder="little").view("<u4")
    return torch.from_numpy(np.ascontiguousarray(words.reshape(-1))).to(device())


@pytest.mark.parametrize("m,n,r,k,p_obs", [(333, 77, 3, 5, 0.6), (1000, 300, 12, 20, 0.4)])
def test_device_mask_context_matches_host_mask_context(m, n, r, k, p_obs):
    p = synth.partial_rpca(m=m, n=n, r=r, k=k, p_obs=p_obs, seed=900 + m)
    dev = device()
    Xcm = T.to_device_X(p.X, dev)
    bits = _pack_mask_dirty(p.mask)
    ch = T.Context(p.m, p.n, p.k, p.lam_s, p.lam_l, p.mask)
    cd = T.Context(p.m, p.n, p.k, p.lam_s, p.lam_l, mask_bits=bits)
    U, V = synth.random_factors(p.m, p.n, p.k, 3, scale=0.4)
    Ud, Vd = T.to_device_factor(U, dev), T.to_device_factor(V, dev)
    fh, gUh, gVh = ch.objgrad(Xcm, Ud, Vd)
    fd, gUd, gVd = cd.objgrad(Xcm, Ud, Vd)
    torch.cuda.synchronize()
    assert fh.item() == fd.item() and torch.equal(gUh, gUd) and torch.equal(gVh, gVd)
    fr, gUr, gVr = ob.objgrad(f32(U), f32(V), f32(p.X), p.lam_s, p.lam_l, p.mask)
    assert abs(fd.item() - fr) <= 1e-5 * abs(fr)
    assert rel(gUd.cpu().numpy(), gUr) <= 1e-5 and rel(gVd.cpu().numpy(), gVr) <= 1e-5
    outs = []
    for c in (ch, cd):
        Us = torch.empty(p.m, p.k, dtype=torch.float32, device=dev)
        Vs = torch.empty(p.n, p.k, dtype=torch.float32, device=dev)
        rc, info = c.solve(Xcm, Us, Vs, init=R.RPCA_INIT_RSVD, certify=1, seed=5)
        torch.cuda.synchronize()
        outs.append((rc, info.iters, info.f, info.rel_gap, Us.cpu(), Vs.cpu()))
    a, b = outs
    print(f"[device mask {m}x{n} k={k}] host rc={a[0]} it={a[1]} f={a[2]:.10g} gap={a[3]:.3e} | "
          f"device rc={b[0]} it={b[1]} f={b[2]:.10g} gap={b[3]:.3e}", flush=True)
    assert a[:4] == b[:4] and torch.equal(a[4], b[4]) and torch.equal(a[5], b[5])
    assert b[0] == R.RPCA_OK and b[3] <= 1e-3
    ch.close()
    cd.close()

