"""Wrappers that take torch device tensors and call the C ABI.

torch provides device memory and the current HIP stream; all arithmetic runs
in librpca.  Shapes: X (m, n) float32 stored column-major (pass ``X_cm``, an
(n, m) contiguous tensor whose rows are the columns of X, or use ``to_device_X``),
U (m, k) and V (n, k) float32 row-major contiguous.
"""
import numpy as np
import torch

from . import rpca as R


def _stream():
    return torch.cuda.current_stream().cuda_stream


def to_device_X(X, device="cuda"):
    """Column-major FP32 copy of a host matrix: an (n, m) tensor whose row j is column j of X."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(X, np.float32).T)).to(device)


def to_device_factor(A, device="cuda"):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A, np.float32))).to(device)


class Context:
    """Owns an rpca_ctx for one problem shape."""

    def __init__(self, m, n, k, lam_s, lam_l, mask=None):
        rc, self.ctx = R.rpca_create(m, n, k, lam_s, lam_l, mask)
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_create failed: {R.rpca_status_string(rc)}")
        self.m, self.n, self.k = m, n, k

    def close(self):
        if self.ctx:
            R.rpca_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def objgrad(self, Xcm, U, V, precision=R.RPCA_PREC_FP32):
        f = torch.empty(1, dtype=torch.float64, device=U.device)
        gU = torch.empty_like(U)
        gV = torch.empty_like(V)
        rc = R.rpca_objgrad_ex(self.ctx, Xcm.data_ptr(), U.data_ptr(), V.data_ptr(), f.data_ptr(),
                               gU.data_ptr(), gV.data_ptr(), precision, _stream())
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_objgrad failed: {R.rpca_status_string(rc)}")
        return f, gU, gV

    def solve(self, Xcm, U, V, **opts):
        o = R.default_opts()
        for key, val in opts.items():
            setattr(o, key, val)
        rc, info = R.rpca_solve(self.ctx, Xcm.data_ptr(), U.data_ptr(), V.data_ptr(), o, _stream())
        if rc < 0:
            raise RuntimeError(f"rpca_solve failed: {R.rpca_status_string(rc)}")
        return rc, info

    def certificate(self, Xcm, U, V):
        rc, cert = R.rpca_certificate(self.ctx, Xcm.data_ptr(), U.data_ptr(), V.data_ptr(), _stream())
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_certificate failed: {R.rpca_status_string(rc)}")
        return cert

    def init_rsvd(self, Xcm, Omega=None, oversample=10, power_steps=2, seed=12345):
        U = torch.empty(self.m, self.k, dtype=torch.float32, device=Xcm.device)
        V = torch.empty(self.n, self.k, dtype=torch.float32, device=Xcm.device)
        om = Omega.data_ptr() if Omega is not None else None
        if Omega is not None:
            oversample = Omega.shape[1] - self.k
        rc = R.rpca_init_rsvd(self.ctx, Xcm.data_ptr(), om, oversample, power_steps, seed,
                              U.data_ptr(), V.data_ptr(), _stream())
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_init_rsvd failed: {R.rpca_status_string(rc)}")
        return U, V
