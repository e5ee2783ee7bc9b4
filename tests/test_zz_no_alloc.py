"""GPU test of rpca_objgrad_noalloc, the objective/gradient entry point that
allocates nothing (its partial sums live in a fixed device array per GPU).

It must give what rpca_objgrad gives on a context of the same sizes -- the
same kernels and decomposition, so bitwise -- and match the FP64 oracle to the
FP32 bar (f and gradients within 1e-5 relative).  Two calls in a row share the
array: the second, on a smaller instance, must not see the first's partials.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import objective as ob
from paper_1702_02241_amd import rpca as R
from paper_1702_02241_amd import synth
from paper_1702_02241_amd import torch_api as T

from gpu_common import device, f32, rel

pytestmark = pytest.mark.gpu


def _pack_mask(mask):
    """Column-major device bitmask: bit i % 32 of word j*ceil(m/32) + i/32."""
    m, n = mask.shape
    mw = (m + 31) // 32
    cols = np.zeros((n, mw * 32), np.uint8)
    cols[:, :m] = (np.asarray(mask) != 0).T
    words = np.packbits(cols, axis=1, bitorder="little").view("<u4")
    return torch.from_numpy(np.ascontiguousarray(words.reshape(-1))).to(device())


def _noalloc(p, Xcm, Ud, Vd, mask_dev):
    f = torch.full((1,), float("nan"), dtype=torch.float64, device=device())
    gU = torch.full_like(Ud, float("nan"))
    gV = torch.full_like(Vd, float("nan"))
    mptr = mask_dev.data_ptr() if mask_dev is not None else None
    rc = R.rpca_objgrad_noalloc(p.m, p.n, p.k, p.lam_s, p.lam_l, mptr, Xcm.data_ptr(),
                                Ud.data_ptr(), Vd.data_ptr(), f.data_ptr(), gU.data_ptr(),
                                gV.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == R.RPCA_OK, R.rpca_status_string(rc)
    return f, gU, gV


def _case(p, seed):
    dev = device()
    U, V = synth.random_factors(p.m, p.n, p.k, seed, scale=0.4)
    Xcm = T.to_device_X(p.X, dev)
    Ud, Vd = T.to_device_factor(U, dev), T.to_device_factor(V, dev)
    mask_dev = _pack_mask(p.mask) if p.mask is not None else None
    f, gU, gV = _noalloc(p, Xcm, Ud, Vd, mask_dev)
    ctx = T.Context(p.m, p.n, p.k, p.lam_s, p.lam_l, p.mask)
    fc, gUc, gVc = ctx.objgrad(Xcm, Ud, Vd)
    torch.cuda.synchronize()
    ctx.close()
    fr, gUr, gVr = ob.objgrad(f32(U), f32(V), f32(p.X), p.lam_s, p.lam_l, p.mask)
    ef = abs(f.item() - fr) / abs(fr)
    eu, ev = rel(gU.cpu().numpy(), gUr), rel(gV.cpu().numpy(), gVr)
    same = (f.item() == fc.item() and torch.equal(gU, gUc) and torch.equal(gV, gVc))
    print(f"[noalloc m={p.m} n={p.n} k={p.k} mask={p.mask is not None}] f rel {ef:.2e} "
          f"gU rel {eu:.2e} gV rel {ev:.2e} bitwise-equal-to-context={same}", flush=True)
    assert same
    assert ef <= 1e-5 and eu <= 1e-5 and ev <= 1e-5


@pytest.mark.parametrize("masked", [False, True])
def test_noalloc_matches_context_and_oracle_on_two_calls(masked):
    if masked:
        big = synth.partial_rpca(m=1500, n=420, r=8, k=12, p_obs=0.4, seed=41)
        small = synth.partial_rpca(m=301, n=77, r=4, k=5, p_obs=0.6, seed=42)
    else:
        big = synth.gaussian_rpca(m=4099, n=513, r=5, k=25, seed=43)   # several chunks, ragged
        small = synth.gaussian_rpca(m=256, n=200, r=5, k=10, seed=44)  # the small Gaussian case
    _case(big, 3)
    _case(small, 4)   # second call on the same array, smaller instance


def test_noalloc_video_full_size():
    p = synth.video()                 # 76,800 x 200, k = 10
    _case(p, 31)


def test_noalloc_rejects_oversize_before_launch():
    # 2^22 x 2^14, k = 32 spans many column chunks: its G V partials need far more
    # than the fixed array; rejected before any device work
    dummy = ctypes.c_void_p(16)
    rc = R.rpca_objgrad_noalloc(1 << 22, 1 << 14, 32, 0.1, 1.0, None, dummy, dummy, dummy,
                                dummy, dummy, dummy, None)
    assert rc == R.RPCA_ETOOBIG
