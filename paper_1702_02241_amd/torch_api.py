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

    def __init__(self, m, n, k, lam_s, lam_l, mask=None, waves=None, mu=0.0, mask_bits=None):
        """mask: host array (m x n, nonzero = observed); or mask_bits: a device tensor
        holding the packed bitmask (int32/uint32 words, column-major, 32 rows a word)."""
        if mask_bits is not None:
            rc, self.ctx = R.rpca_create_device_mask(m, n, k, lam_s, lam_l, mask_bits.data_ptr(), waves or 0)
        else:
            rc, self.ctx = R.rpca_create(m, n, k, lam_s, lam_l, mask, waves)
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_create failed: {R.rpca_status_string(rc)}")
        self.m, self.n, self.k = m, n, k
        if mu:
            self.set_elastic(mu)

    def set_elastic(self, mu):
        """Elastic-net regulariser lam_s ||S||_1 + mu/2 ||S||_F^2 (mu = 0: l1)."""
        rc = R.lib().rpca_set_elastic(self.ctx, float(mu))
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_set_elastic failed: {R.rpca_status_string(rc)}")

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

    def prox_solve(self, Xcm, max_iter=500, tol=1e-8, oversample=10, power_steps=1, seed=7):
        """Convex baseline (accelerated proximal gradient with randomized SVT from L = 0).
        Returns (status, info, U (m, k), V (n, k)), L = U V^T."""
        U = torch.empty(self.m, self.k, dtype=torch.float32, device=Xcm.device)
        V = torch.empty(self.n, self.k, dtype=torch.float32, device=Xcm.device)
        rc, info = R.rpca_prox_solve(self.ctx, Xcm.data_ptr(), U.data_ptr(), V.data_ptr(), max_iter, tol, oversample,
                                     power_steps, seed, _stream())
        if rc < 0:
            raise RuntimeError(f"rpca_prox_solve failed: {R.rpca_status_string(rc)}")
        return rc, info, U, V

    def rank_direction(self, Xcm, U, V):
        """Growth column pair at L = U V^T: (sigma, t, u_col (m,), v_col (n,))."""
        u_col = torch.empty(self.m, dtype=torch.float32, device=U.device)
        v_col = torch.empty(self.n, dtype=torch.float32, device=U.device)
        rc, sigma, t = R.rpca_rank_direction(self.ctx, Xcm.data_ptr(), U.data_ptr(), V.data_ptr(),
                                             u_col.data_ptr(), v_col.data_ptr(), _stream())
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_rank_direction failed: {R.rpca_status_string(rc)}")
        return sigma, t, u_col, v_col

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


def solve_grow(Xcm, m, n, k0, k_max, lam_s, lam_l, mask=None, U0=None, V0=None, **opts):
    """Solve with the rank grown from k0 up to k_max on demand (rpca_solve_grow).
    U0, V0: (m, k0), (n, k0) start, or None for the randomized-SVD start.
    Returns (status, info, U (m, k), V (n, k))."""
    o = R.default_opts()
    for key, val in opts.items():
        setattr(o, key, val)
    Ub = torch.zeros(m * k_max, dtype=torch.float32, device=Xcm.device)
    Vb = torch.zeros(n * k_max, dtype=torch.float32, device=Xcm.device)
    if U0 is None:
        o.init = R.RPCA_INIT_RSVD
    else:
        Ub[: m * k0].copy_(U0.reshape(-1))
        Vb[: n * k0].copy_(V0.reshape(-1))
    rc, k, info = R.rpca_solve_grow(m, n, k0, k_max, lam_s, lam_l, mask, Xcm.data_ptr(), Ub.data_ptr(),
                                    Vb.data_ptr(), o, _stream())
    if rc < 0:
        raise RuntimeError(f"rpca_solve_grow failed: {R.rpca_status_string(rc)}")
    return rc, info, Ub[: m * k].view(m, k), Vb[: n * k].view(n, k)


class FrankWolfe:
    """Owns an rpca_fw (rpca_fw.h): Frank-Wolfe with the sparse part marginalised.
    L lives as an (n, m) contiguous tensor, the column-major layout of X_cm."""

    def __init__(self, m, n, lam_s, lam_l, mask=None):
        rc, self.h = R.rpca_fw_create(m, n, lam_s, lam_l, mask)
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_fw_create failed: {R.rpca_status_string(rc)}")
        self.m, self.n = m, n

    def close(self):
        if self.h:
            R.rpca_fw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, on):
        R.lib().rpca_fw_profile_enable(self.h, 1 if on else 0)

    def profile_read(self, reset=True):
        rc, launches, ms = R.rpca_fw_profile_read(self.h, reset)
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_fw_profile_read failed: {R.rpca_status_string(rc)}")
        return launches, ms

    def solve(self, Xcm, Lcm=None, t=0.0, max_iter=1000, tol=1e-6, power_tol=0.0):
        """Returns (status, Lcm, t, info); Lcm None starts from L = 0, t = 0."""
        if Lcm is None:
            Lcm = torch.zeros_like(Xcm)
            t = 0.0
        rc, t, info = R.rpca_fw_solve(self.h, Xcm.data_ptr(), Lcm.data_ptr(), t, max_iter, tol, power_tol,
                                      _stream())
        if rc < 0:
            raise RuntimeError(f"rpca_fw_solve failed: {R.rpca_status_string(rc)}")
        return rc, Lcm, t, info


class WarmNet:
    """Owns an rpca_mlp (rpca_warm.h): the 2-layer warm-start network."""

    def __init__(self, d_in, d_h, mu, nv, k, max_batch=64, seed=0):
        rc, self.net = R.rpca_mlp_create(d_in, d_h, mu, nv, k, max_batch, seed)
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_mlp_create failed: {R.rpca_status_string(rc)}")
        self.d_in, self.d_h, self.mu, self.nv, self.k = d_in, d_h, mu, nv, k
        self.d_out = (mu + nv) * k
        self.max_batch = max_batch

    def close(self):
        if self.net:
            R.rpca_mlp_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, W1, b1, W2, b2):
        """Overwrite the parameters from host arrays (float32 copies)."""
        for which, arr in enumerate((W1, b1, W2, b2)):
            rc, ptr, cnt = R.rpca_mlp_param(self.net, which)
            a = np.ascontiguousarray(np.asarray(arr, np.float32)).reshape(-1)
            if a.size != cnt:
                raise ValueError("parameter shape mismatch")
            _copy_host_to_device(ptr, a)

    def params(self):
        return [_copy_device_to_host(*R.rpca_mlp_param(self.net, w)[1:]) for w in range(4)]

    def grads(self):
        return [_copy_device_to_host(*R.rpca_mlp_grad(self.net, w)[1:]) for w in range(4)]

    def forward(self, x):
        y = torch.empty(x.shape[0], self.d_out, dtype=torch.float32, device=x.device)
        rc = R.rpca_mlp_forward(self.net, x.data_ptr(), x.shape[0], y.data_ptr(), _stream())
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_mlp_forward failed: {R.rpca_status_string(rc)}")
        return y

    def loss_grad(self, x, TU, TV):
        loss = torch.empty(1, dtype=torch.float64, device=x.device)
        rc = R.rpca_mlp_loss_grad(self.net, x.data_ptr(), TU.data_ptr(), TV.data_ptr(), x.shape[0],
                                  loss.data_ptr(), _stream())
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_mlp_loss_grad failed: {R.rpca_status_string(rc)}")
        return loss

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        rc = R.rpca_mlp_adam_step(self.net, lr, beta1, beta2, eps, _stream())
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_mlp_adam_step failed: {R.rpca_status_string(rc)}")

    def train_step(self, x, TU, TV, lr):
        loss = torch.empty(1, dtype=torch.float64, device=x.device)
        rc = R.rpca_mlp_train_step(self.net, x.data_ptr(), TU.data_ptr(), TV.data_ptr(), x.shape[0], lr,
                                   loss.data_ptr(), _stream())
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_mlp_train_step failed: {R.rpca_status_string(rc)}")
        return loss


def _hip():
    """The HIP runtime already loaded by torch and librpca (same soname)."""
    import ctypes
    h = ctypes.CDLL("libamdhip64.so.7")
    h.hipMemcpy.restype = ctypes.c_int
    h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return h


def _copy_host_to_device(ptr, a):
    """Copy a contiguous float32 host array into library-owned device memory (synchronous)."""
    torch.cuda.synchronize()
    if _hip().hipMemcpy(ptr, a.ctypes.data, a.nbytes, 1) != 0:
        raise RuntimeError("hipMemcpy host->device failed")


def _copy_device_to_host(ptr, count):
    torch.cuda.synchronize()
    out = np.empty(count, np.float32)
    if _hip().hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2) != 0:
        raise RuntimeError("hipMemcpy device->host failed")
    return out


def window_features(Xcm_window, width, height, frames, factor, shift=None, scale=None):
    """Features of one window: Xcm_window is a (frames, width*height) contiguous
    device tensor (column-major X of the window).  Returns a d_in device vector."""
    mu = (width // factor) * (height // factor)
    feat = torch.empty(2 * mu + frames, dtype=torch.float32, device=Xcm_window.device)
    rc = R.rpca_window_features(Xcm_window.data_ptr(), width, height, frames, factor,
                                shift.data_ptr() if shift is not None else None,
                                scale.data_ptr() if scale is not None else None, feat.data_ptr(), _stream())
    if rc != R.RPCA_OK:
        raise RuntimeError(f"rpca_window_features failed: {R.rpca_status_string(rc)}")
    return feat


def pool_rows(A, width, height, factor):
    c = A.shape[1]
    out = torch.empty((width // factor) * (height // factor), c, dtype=torch.float32, device=A.device)
    rc = R.rpca_pool_rows(A.data_ptr(), width, height, factor, c, out.data_ptr(), _stream())
    if rc != R.RPCA_OK:
        raise RuntimeError(f"rpca_pool_rows failed: {R.rpca_status_string(rc)}")
    return out


def upsample_rows(A, width, height, factor):
    c = A.shape[1]
    out = torch.empty(width * height, c, dtype=torch.float32, device=A.device)
    rc = R.rpca_upsample_rows(A.data_ptr(), width, height, factor, c, out.data_ptr(), _stream())
    if rc != R.RPCA_OK:
        raise RuntimeError(f"rpca_upsample_rows failed: {R.rpca_status_string(rc)}")
    return out


class Batch:
    """Owns an rpca_batch (rpca_batch.h) for a list of fully observed instances."""

    def __init__(self, shapes, lam_s, lam_l):
        """shapes: list of (m, n, k); lam_s, lam_l: sequences of per-instance weights."""
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        m, n, k = zip(*self.shapes)
        rc, self.b = R.rpca_batch_create(m, n, k, list(lam_s), list(lam_l))
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_batch_create failed: {R.rpca_status_string(rc)}")

    def close(self):
        if self.b:
            R.rpca_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graphs(self, on):
        R.rpca_batch_set_graphs(self.b, on)

    def layout(self):
        return R.rpca_batch_info(self.b)[1]

    def instance_waves(self, i):
        rc, w = R.rpca_batch_instance_waves(self.b, i)
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_batch_instance_waves failed: {R.rpca_status_string(rc)}")
        return w

    def objgrad(self, Xs, Us, Vs, precision=R.RPCA_PREC_FP32):
        dev = Us[0].device
        fs = [torch.empty(1, dtype=torch.float64, device=dev) for _ in Us]
        gUs = [torch.empty_like(U) for U in Us]
        gVs = [torch.empty_like(V) for V in Vs]
        rc = R.rpca_batch_objgrad(self.b, [x.data_ptr() for x in Xs], [u.data_ptr() for u in Us],
                                  [v.data_ptr() for v in Vs], [f.data_ptr() for f in fs],
                                  [g.data_ptr() for g in gUs], [g.data_ptr() for g in gVs], precision, _stream())
        if rc != R.RPCA_OK:
            raise RuntimeError(f"rpca_batch_objgrad failed: {R.rpca_status_string(rc)}")
        return fs, gUs, gVs

    def solve(self, Xs, Us, Vs, **opts):
        o = R.default_opts()
        for key, val in opts.items():
            setattr(o, key, val)
        rc, infos = R.rpca_batch_solve(self.b, [x.data_ptr() for x in Xs], [u.data_ptr() for u in Us],
                                       [v.data_ptr() for v in Vs], o, _stream())
        if rc < 0:
            raise RuntimeError(f"rpca_batch_solve failed: {R.rpca_status_string(rc)}")
        return rc, infos
