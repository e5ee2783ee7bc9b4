"""ctypes binding of librpca (the C ABI in include/rpca.h).

Argument marshalling only: every step of the method runs inside the HIP
library.  Device buffers are passed as integer addresses (``tensor.data_ptr()``)
and streams as ``torch.cuda.current_stream().cuda_stream``; torch is only the
allocator and stream provider.  Loading fails loudly when the library has not
been built -- there is no CPU fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpca.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "rpca.h")
HEADER_PATHS = [HEADER_PATH, os.path.join(os.path.dirname(HEADER_PATH), "rpca_warm.h"),
                os.path.join(os.path.dirname(HEADER_PATH), "rpca_batch.h"),
                os.path.join(os.path.dirname(HEADER_PATH), "rpca_fw.h")]

RPCA_OK, RPCA_ENOTCONV, RPCA_ELINESEARCH, RPCA_ENOTCERT = 0, 1, 2, 3
RPCA_EINVAL, RPCA_ENOMEM, RPCA_EHIP, RPCA_ENONFINITE, RPCA_ETOOBIG = -1, -2, -3, -4, -5
RPCA_PREC_FP32, RPCA_PREC_BF16_POLISH, RPCA_PREC_BF16 = 0, 1, 2
RPCA_INIT_GIVEN, RPCA_INIT_RSVD = 0, 1


class rpca_opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("mem", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("init", ctypes.c_int32),
        ("gtol", ctypes.c_double),
        ("ftol", ctypes.c_double),
        ("bf16_gtol", ctypes.c_double),
        ("c1", ctypes.c_double),
        ("c2", ctypes.c_double),
        ("certify", ctypes.c_int32),
        ("cert_tol", ctypes.c_double),
        ("rsvd_oversample", ctypes.c_int32),
        ("rsvd_power", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("slots_per_sync", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("precond_cycle", ctypes.c_int32),
    ]


class rpca_info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("evals", ctypes.c_int32),
        ("iters_bf16", ctypes.c_int32),
        ("f", ctypes.c_double),
        ("gnorm_inf", ctypes.c_double),
        ("rel_gap", ctypes.c_double),
        ("certified", ctypes.c_int32),
        ("cert_rounds", ctypes.c_int32),
        ("seconds", ctypes.c_double),
    ]


class rpca_cert(ctypes.Structure):
    _fields_ = [
        ("T1", ctypes.c_double), ("T2", ctypes.c_double), ("T3", ctypes.c_double),
        ("T4", ctypes.c_double), ("E", ctypes.c_double), ("F", ctypes.c_double),
        ("phi", ctypes.c_double), ("phi0", ctypes.c_double), ("F_bound", ctypes.c_double),
        ("normL", ctypes.c_double), ("gap", ctypes.c_double), ("rel_gap", ctypes.c_double),
        ("normM2", ctypes.c_double),
        ("theta", ctypes.c_double * 32),
        ("sigma", ctypes.c_double * 64),
        ("r", ctypes.c_int32), ("power_iters", ctypes.c_int32), ("block", ctypes.c_int32),
        ("certified", ctypes.c_int32),
    ]


class rpca_prox_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("rank", ctypes.c_int32), ("sketch", ctypes.c_int32), ("truncated", ctypes.c_int32),
                ("F", ctypes.c_double), ("rel_change", ctypes.c_double), ("seconds", ctypes.c_double)]


class rpca_fw_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("power_iters", ctypes.c_int32),
                ("last_step", ctypes.c_int32), ("F", ctypes.c_double), ("phi", ctypes.c_double),
                ("gap", ctypes.c_double), ("sigma", ctypes.c_double), ("eta", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class rpca_batch_layout(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("sweep_items", ctypes.c_int32),
                ("sweep_grid_fp32", ctypes.c_int32), ("sweep_grid_bf16", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("graphs", ctypes.c_int32),
                ("sweep_classes", ctypes.c_int32)]


class rpca_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 8), ("ms", ctypes.c_double * 8)]


class rpca_fw_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 4), ("ms", ctypes.c_double * 4)]


RPCA_K_SWEEP, RPCA_K_FINISH, RPCA_K_UPDATE, RPCA_K_DIRECTION, RPCA_K_TRIAL, RPCA_K_LEFT, RPCA_K_RIGHT = 0, 1, 2, 3, 4, 5, 6
RPCA_K_GRAM = 7

_lib = None


def lib():
    """Load librpca.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1702_02241_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        sig = {
            "rpca_default_opts": (None, [ctypes.POINTER(rpca_opts)]),
            "rpca_create": (I32, [I64, I64, I32, D, D, P, ctypes.POINTER(P)]),
            "rpca_create_waves": (I32, [I64, I64, I32, D, D, P, I32, ctypes.POINTER(P)]),
            "rpca_create_device_mask": (I32, [I64, I64, I32, D, D, P, I32, ctypes.POINTER(P)]),
            "rpca_objgrad": (I32, [P, P, P, P, P, P, P, P]),
            "rpca_set_elastic": (I32, [P, D]),
            "rpca_sweep_layout": (I32, [P, ctypes.POINTER(I32 * 4)]),
            "rpca_set_graphs": (I32, [P, I32]),
            "rpca_objgrad_ex": (I32, [P, P, P, P, P, P, P, I32, P]),
            "rpca_objgrad_noalloc": (I32, [I64, I64, I32, D, D, P, P, P, P, P, P, P, P]),
            "rpca_solve": (I32, [P, P, P, P, ctypes.POINTER(rpca_opts), ctypes.POINTER(rpca_info), P]),
            "rpca_certificate": (I32, [P, P, P, P, ctypes.POINTER(rpca_cert), P]),
            "rpca_rank_direction": (I32, [P, P, P, P, P, P, ctypes.POINTER(D), ctypes.POINTER(D), P]),
            "rpca_solve_grow": (I32, [I64, I64, I32, I32, D, D, P, P, P, P, ctypes.POINTER(I32),
                                      ctypes.POINTER(rpca_opts), ctypes.POINTER(rpca_info), P]),
            "rpca_init_rsvd": (I32, [P, P, P, I32, I32, U64, P, P, P]),
            "rpca_prox_solve": (I32, [P, P, P, P, I32, D, I32, I32, U64, ctypes.POINTER(rpca_prox_info), P]),
            "rpca_destroy": (None, [P]),
            "rpca_status_string": (ctypes.c_char_p, [I32]),
            "rpca_profile_enable": (I32, [P, I32]),
            "rpca_profile_read": (I32, [P, ctypes.POINTER(rpca_profile), I32]),
            # learned warm start (rpca_warm.h)
            "rpca_mlp_create": (I32, [I32, I32, I32, I32, I32, I32, U64, ctypes.POINTER(P)]),
            "rpca_mlp_param": (I32, [P, I32, ctypes.POINTER(P), ctypes.POINTER(I64)]),
            "rpca_mlp_grad": (I32, [P, I32, ctypes.POINTER(P), ctypes.POINTER(I64)]),
            "rpca_mlp_forward": (I32, [P, P, I32, P, P]),
            "rpca_mlp_loss_grad": (I32, [P, P, P, P, I32, P, P]),
            "rpca_mlp_adam_step": (I32, [P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, P]),
            "rpca_mlp_train_step": (I32, [P, P, P, P, I32, ctypes.c_float, P, P]),
            "rpca_mlp_destroy": (None, [P]),
            "rpca_window_features": (I32, [P, I64, I64, I32, I32, P, P, P, P]),
            "rpca_pool_rows": (I32, [P, I64, I64, I32, I32, P, P]),
            "rpca_upsample_rows": (I32, [P, I64, I64, I32, I32, P, P]),
            # batched instances (rpca_batch.h)
            "rpca_batch_create": (I32, [I32, P, P, P, P, P, ctypes.POINTER(P)]),
            "rpca_batch_objgrad": (I32, [P, P, P, P, P, P, P, I32, P]),
            "rpca_batch_solve": (I32, [P, P, P, P, ctypes.POINTER(rpca_opts), P, P]),
            "rpca_batch_set_graphs": (I32, [P, I32]),
            "rpca_batch_info": (I32, [P, ctypes.POINTER(rpca_batch_layout)]),
            "rpca_batch_instance_waves": (I32, [P, I32, ctypes.POINTER(I32)]),
            "rpca_batch_destroy": (None, [P]),
            "rpca_autotune": (I32, [I64, I32, P]),
            # Frank-Wolfe with marginalisation (rpca_fw.h)
            "rpca_fw_create": (I32, [I64, I64, D, D, P, ctypes.POINTER(P)]),
            "rpca_fw_solve": (I32, [P, P, P, ctypes.POINTER(D), I32, D, D, ctypes.POINTER(rpca_fw_info), P]),
            "rpca_fw_destroy": (None, [P]),
            "rpca_fw_profile_enable": (I32, [P, I32]),
            "rpca_fw_profile_read": (I32, [P, ctypes.POINTER(rpca_fw_profile), I32]),
            "rpca_tune_get": (I32, [I32, I64, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
            "rpca_tune_set": (I32, [I32, I64, I32, I32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def default_opts():
    o = rpca_opts()
    lib().rpca_default_opts(ctypes.byref(o))
    return o


def rpca_create_device_mask(m, n, k, lam_s, lam_l, mask_bits_ptr, waves=0):
    """mask_bits_ptr: device address of the packed bitmask (column-major words of 32
    rows).  Returns (status, ctx)."""
    ctx = ctypes.c_void_p()
    rc = lib().rpca_create_device_mask(m, n, k, lam_s, lam_l, mask_bits_ptr, int(waves), ctypes.byref(ctx))
    return rc, ctx


def rpca_create(m, n, k, lam_s, lam_l, mask=None, waves=None):
    """mask: None or a host numpy uint8 array (m x n, Fortran order or any order;
    it is converted to column-major bytes).  waves: None (rpca_create) or the
    sweep's wave target (rpca_create_waves).  Returns (status, ctx)."""
    ctx = ctypes.c_void_p()
    mptr = None
    keep = None
    if mask is not None:
        import numpy as np
        keep = np.asfortranarray(np.asarray(mask) != 0, dtype=np.uint8)
        mptr = keep.ctypes.data
    if waves is None:
        rc = lib().rpca_create(m, n, k, lam_s, lam_l, mptr, ctypes.byref(ctx))
    else:
        rc = lib().rpca_create_waves(m, n, k, lam_s, lam_l, mptr, int(waves), ctypes.byref(ctx))
    return rc, ctx


def rpca_set_graphs(ctx, on):
    return lib().rpca_set_graphs(ctx, int(on))


def rpca_sweep_layout(ctx):
    """(status, (workgroup rows, strips per wave, chunk columns, chunks))."""
    out = (ctypes.c_int32 * 4)()
    rc = lib().rpca_sweep_layout(ctx, ctypes.byref(out))
    return rc, tuple(out)


def rpca_objgrad(ctx, X, U, V, f, gU, gV, stream=0):
    return lib().rpca_objgrad(ctx, X, U, V, f, gU, gV, stream)


def rpca_objgrad_ex(ctx, X, U, V, f, gU, gV, precision, stream=0):
    return lib().rpca_objgrad_ex(ctx, X, U, V, f, gU, gV, precision, stream)


def rpca_objgrad_noalloc(m, n, k, lam_s, lam_l, mask_bits, X, U, V, f, gU, gV, stream=0):
    return lib().rpca_objgrad_noalloc(m, n, k, lam_s, lam_l, mask_bits, X, U, V, f, gU, gV, stream)


def rpca_solve(ctx, X, U, V, opts=None, stream=0):
    info = rpca_info()
    rc = lib().rpca_solve(ctx, X, U, V, ctypes.byref(opts) if opts is not None else None,
                          ctypes.byref(info), stream)
    return rc, info


def rpca_certificate(ctx, X, U, V, stream=0):
    cert = rpca_cert()
    rc = lib().rpca_certificate(ctx, X, U, V, ctypes.byref(cert), stream)
    return rc, cert


def rpca_rank_direction(ctx, X, U, V, u_col, v_col, stream=0):
    """Growth column pair (device u_col: m, v_col: n floats).  Returns
    (status, sigma, t)."""
    sigma, t = ctypes.c_double(), ctypes.c_double()
    rc = lib().rpca_rank_direction(ctx, X, U, V, u_col, v_col, ctypes.byref(sigma), ctypes.byref(t), stream)
    return rc, sigma.value, t.value


def rpca_solve_grow(m, n, k0, k_max, lam_s, lam_l, mask, X, U, V, opts=None, stream=0):
    """Solve with the rank grown on demand.  mask: None or host array (as
    rpca_create).  U, V: device buffers of m*k_max, n*k_max floats.  Returns
    (status, k, info)."""
    info = rpca_info()
    k = ctypes.c_int32()
    mptr = None
    keep = None
    if mask is not None:
        import numpy as np
        keep = np.asfortranarray(np.asarray(mask) != 0, dtype=np.uint8)
        mptr = keep.ctypes.data
    rc = lib().rpca_solve_grow(m, n, k0, k_max, lam_s, lam_l, mptr, X, U, V, ctypes.byref(k),
                               ctypes.byref(opts) if opts is not None else None, ctypes.byref(info),
                               stream)
    del keep
    return rc, k.value, info


def rpca_fw_create(m, n, lam_s, lam_l, mask=None):
    """mask: None or host array (m x n, any order; converted to column-major bytes).
    Returns (status, handle)."""
    h = ctypes.c_void_p()
    mptr = None
    keep = None
    if mask is not None:
        import numpy as np
        keep = np.asfortranarray(np.asarray(mask) != 0, dtype=np.uint8)
        mptr = keep.ctypes.data
    rc = lib().rpca_fw_create(m, n, lam_s, lam_l, mptr, ctypes.byref(h))
    del keep
    return rc, h


def rpca_fw_solve(h, X, L, t, max_iter, tol, power_tol=0.0, stream=0):
    """Returns (status, t, info)."""
    tt = ctypes.c_double(t)
    info = rpca_fw_info()
    rc = lib().rpca_fw_solve(h, X, L, ctypes.byref(tt), max_iter, tol, power_tol, ctypes.byref(info), stream)
    return rc, tt.value, info


def rpca_fw_destroy(h):
    lib().rpca_fw_destroy(h)


RPCA_FW_K_UPDATE, RPCA_FW_K_LEFT, RPCA_FW_K_RIGHT, RPCA_FW_K_BILINEAR = 0, 1, 2, 3


def rpca_fw_profile_read(h, reset=True):
    """(status, launches[4], ms[4]) per kernel class."""
    p = rpca_fw_profile()
    rc = lib().rpca_fw_profile_read(h, ctypes.byref(p), 1 if reset else 0)
    return rc, list(p.launches), list(p.ms)


def rpca_prox_solve(ctx, X, U, V, max_iter=500, tol=1e-8, oversample=10, power_steps=1, seed=7, stream=0):
    """Returns (status, info)."""
    info = rpca_prox_info()
    rc = lib().rpca_prox_solve(ctx, X, U, V, max_iter, tol, oversample, power_steps, seed, ctypes.byref(info),
                               stream)
    return rc, info


def rpca_init_rsvd(ctx, X, Omega, oversample, power_steps, seed, U, V, stream=0):
    return lib().rpca_init_rsvd(ctx, X, Omega, oversample, power_steps, seed, U, V, stream)


def rpca_destroy(ctx):
    lib().rpca_destroy(ctx)


def rpca_status_string(status):
    return lib().rpca_status_string(status).decode()


def rpca_profile_enable(ctx, on):
    return lib().rpca_profile_enable(ctx, 1 if on else 0)


def rpca_profile_read(ctx, reset=False):
    prof = rpca_profile()
    rc = lib().rpca_profile_read(ctx, ctypes.byref(prof), 1 if reset else 0)
    return rc, prof


RPCA_MLP_W1, RPCA_MLP_B1, RPCA_MLP_W2, RPCA_MLP_B2 = 0, 1, 2, 3


def rpca_mlp_create(d_in, d_h, mu, nv, k, max_batch, seed):
    net = ctypes.c_void_p()
    rc = lib().rpca_mlp_create(d_in, d_h, mu, nv, k, max_batch, seed, ctypes.byref(net))
    return rc, net


def rpca_mlp_param(net, which):
    ptr, cnt = ctypes.c_void_p(), ctypes.c_int64()
    rc = lib().rpca_mlp_param(net, which, ctypes.byref(ptr), ctypes.byref(cnt))
    return rc, ptr.value, cnt.value


def rpca_mlp_grad(net, which):
    ptr, cnt = ctypes.c_void_p(), ctypes.c_int64()
    rc = lib().rpca_mlp_grad(net, which, ctypes.byref(ptr), ctypes.byref(cnt))
    return rc, ptr.value, cnt.value


def rpca_mlp_forward(net, x, batch, y, stream=0):
    return lib().rpca_mlp_forward(net, x, batch, y, stream)


def rpca_mlp_loss_grad(net, x, TU, TV, batch, loss, stream=0):
    return lib().rpca_mlp_loss_grad(net, x, TU, TV, batch, loss, stream)


def rpca_mlp_adam_step(net, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=0):
    return lib().rpca_mlp_adam_step(net, lr, beta1, beta2, eps, stream)


def rpca_mlp_train_step(net, x, TU, TV, batch, lr, loss, stream=0):
    return lib().rpca_mlp_train_step(net, x, TU, TV, batch, lr, loss, stream)


def rpca_mlp_destroy(net):
    lib().rpca_mlp_destroy(net)


def rpca_window_features(X, width, height, frames, factor, shift, scale, feat, stream=0):
    return lib().rpca_window_features(X, width, height, frames, factor, shift, scale, feat, stream)


def rpca_pool_rows(A, width, height, factor, c, out, stream=0):
    return lib().rpca_pool_rows(A, width, height, factor, c, out, stream)


def rpca_upsample_rows(A, width, height, factor, c, out, stream=0):
    return lib().rpca_upsample_rows(A, width, height, factor, c, out, stream)


def _ptr_array(ptrs, ctype=ctypes.c_void_p):
    return (ctype * len(ptrs))(*ptrs)


def rpca_batch_create(m, n, k, lam_s, lam_l):
    """Sequences of per-instance sizes and weights.  Returns (status, batch)."""
    cnt = len(m)
    b = ctypes.c_void_p()
    rc = lib().rpca_batch_create(cnt, (ctypes.c_int64 * cnt)(*m), (ctypes.c_int64 * cnt)(*n),
                                 (ctypes.c_int32 * cnt)(*k), (ctypes.c_double * cnt)(*lam_s),
                                 (ctypes.c_double * cnt)(*lam_l), ctypes.byref(b))
    return rc, b


def rpca_batch_objgrad(b, X, U, V, f, gU, gV, precision=0, stream=0):
    """X, U, V, f, gU, gV: sequences of device pointers (ints)."""
    return lib().rpca_batch_objgrad(b, _ptr_array(X), _ptr_array(U), _ptr_array(V), _ptr_array(f),
                                    _ptr_array(gU), _ptr_array(gV), precision, stream)


def rpca_batch_solve(b, X, U, V, opts=None, stream=0):
    cnt = len(X)
    infos = (rpca_info * cnt)()
    rc = lib().rpca_batch_solve(b, _ptr_array(X), _ptr_array(U), _ptr_array(V),
                                ctypes.byref(opts) if opts is not None else None, infos, stream)
    return rc, list(infos)


def rpca_batch_set_graphs(b, on):
    return lib().rpca_batch_set_graphs(b, 1 if on else 0)


def rpca_batch_info(b):
    out = rpca_batch_layout()
    rc = lib().rpca_batch_info(b, ctypes.byref(out))
    return rc, out


def rpca_batch_instance_waves(b, i):
    w = ctypes.c_int32()
    rc = lib().rpca_batch_instance_waves(b, int(i), ctypes.byref(w))
    return rc, w.value


def rpca_batch_destroy(b):
    lib().rpca_batch_destroy(b)


def rpca_autotune(m_probe=16384, reps=10, stream=0):
    return lib().rpca_autotune(m_probe, reps, stream)


def rpca_tune_get(k, n):
    w, d = ctypes.c_int32(), ctypes.c_int32()
    rc = lib().rpca_tune_get(k, n, ctypes.byref(w), ctypes.byref(d))
    return rc, w.value, d.value


def rpca_tune_set(k, n, target_waves, chunk_div):
    return lib().rpca_tune_set(k, n, target_waves, chunk_div)
