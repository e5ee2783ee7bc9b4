"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, fills defaults, and rejects bad arguments before any HIP call
(so these run without a GPU)."""
import ctypes
import re

import pytest

from paper_1702_02241_amd import rpca as R


def _declared_symbols():
    names = set()
    for path in R.HEADER_PATHS:
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(rpca_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = R.lib()
    names = _declared_symbols()
    assert "rpca_create" in names and "rpca_solve" in names and "rpca_certificate" in names
    assert "rpca_mlp_train_step" in names and "rpca_window_features" in names
    for name in names:
        assert hasattr(L, name), f"{name} declared in a header but not exported"


def test_default_opts():
    o = R.default_opts()
    assert o.mem == 10 and o.precision == R.RPCA_PREC_FP32
    assert o.c1 == 1e-4 and o.c2 == 0.9 and o.cert_tol == 1e-3


@pytest.mark.parametrize("args", [
    (0, 10, 2, 0.1, 1.0),      # m < 1
    (10, 0, 2, 0.1, 1.0),      # n < 1
    (10, 10, 0, 0.1, 1.0),     # k < 1
    (10, 10, 33, 0.1, 1.0),    # k > 32
    (10, 5, 6, 0.1, 1.0),      # k > min(m, n)
    (10, 10, 2, 0.0, 1.0),     # lam_s <= 0
    (10, 10, 2, 0.1, -1.0),    # lam_l <= 0
    (10, 10, 2, float("nan"), 1.0),
])
def test_create_rejects_bad_arguments_before_hip(args):
    rc, ctx = R.rpca_create(*args)
    assert rc == R.RPCA_EINVAL
    assert not ctx.value


@pytest.mark.parametrize("waves", [-1, (1 << 20) + 1])
def test_create_waves_rejects_bad_target(waves):
    rc, ctx = R.rpca_create(100, 20, 5, 0.1, 1.0, None, waves)
    assert rc == R.RPCA_EINVAL
    assert not ctx.value
    rc, ctx = R.rpca_create(100, 20, 0, 0.1, 1.0, None, 64)    # k = 0 fails before any HIP call
    assert rc == R.RPCA_EINVAL


def test_null_context_rejected():
    assert R.rpca_objgrad(None, 1, 1, 1, 1, 1, 1, 0) == R.RPCA_EINVAL
    rc, _ = R.rpca_solve(None, 1, 1, 1)
    assert rc == R.RPCA_EINVAL
    rc, _ = R.rpca_certificate(None, 1, 1, 1)
    assert rc == R.RPCA_EINVAL
    assert R.rpca_rank_direction(None, 1, 1, 1, 1, 1)[0] == R.RPCA_EINVAL
    R.rpca_destroy(None)


@pytest.mark.parametrize("k0,k_max,m,n", [(0, 4, 50, 40), (5, 4, 50, 40), (2, 33, 64, 64),
                                          (2, 6, 5, 40), (2, 6, 50, 5)])
def test_solve_grow_rejects_bad_ranks_before_hip(k0, k_max, m, n):
    rc, k, _ = R.rpca_solve_grow(m, n, k0, k_max, 0.1, 1.0, None, 1, 1, 1)
    assert rc == R.RPCA_EINVAL


def test_solve_grow_rejects_null_buffers_and_bad_opts():
    assert R.rpca_solve_grow(50, 40, 2, 4, 0.1, 1.0, None, None, 1, 1)[0] == R.RPCA_EINVAL
    o = R.default_opts()
    o.mem = 0
    assert R.rpca_solve_grow(50, 40, 2, 4, 0.1, 1.0, None, 1, 1, 1, o)[0] == R.RPCA_EINVAL


def test_status_strings():
    assert R.rpca_status_string(R.RPCA_OK) == "ok"
    assert "invalid" in R.rpca_status_string(R.RPCA_EINVAL)


def test_struct_layouts_match_header_order():
    # the ctypes mirrors must list the fields in header order
    text = open(R.HEADER_PATH).read()
    for struct, cls in (("rpca_opts", R.rpca_opts), ("rpca_info", R.rpca_info), ("rpca_cert", R.rpca_cert)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (struct, struct), text, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"(\w+)(?:\[\d+\])?\s*[;,]", body)
        assert [f for f, _ in cls._fields_] == fields


def test_warm_start_entry_points_reject_bad_arguments_before_hip():
    P = ctypes.c_void_p
    net = P()
    L = R.lib()
    assert L.rpca_mlp_create(0, 8, 4, 4, 2, 4, 0, ctypes.byref(net)) == R.RPCA_EINVAL
    assert L.rpca_mlp_create(8, 8, 4, 4, 33, 4, 0, ctypes.byref(net)) == R.RPCA_EINVAL   # k > 32
    assert L.rpca_mlp_create(8, 8, 4, 4, 2, 0, 0, ctypes.byref(net)) == R.RPCA_EINVAL    # batch bound
    assert L.rpca_mlp_create(8, 8, 4, 4, 2, 4097, 0, ctypes.byref(net)) == R.RPCA_EINVAL
    assert not net.value
    assert R.rpca_mlp_forward(None, 1, 1, 1) == R.RPCA_EINVAL
    assert R.rpca_mlp_loss_grad(None, 1, 1, 1, 1, 1) == R.RPCA_EINVAL
    assert R.rpca_mlp_adam_step(None, 1e-3) == R.RPCA_EINVAL
    assert R.rpca_mlp_param(None, 0)[0] == R.RPCA_EINVAL
    # factor must divide the frame; shift and scale come together
    assert R.rpca_window_features(1, 10, 8, 3, 3, None, None, 1) == R.RPCA_EINVAL
    assert R.rpca_window_features(1, 12, 8, 3, 4, 1, None, 1) == R.RPCA_EINVAL
    assert R.rpca_pool_rows(1, 10, 8, 4, 2, 1) == R.RPCA_EINVAL
    assert R.rpca_upsample_rows(1, 12, 8, 4, 0, 1) == R.RPCA_EINVAL
    R.rpca_mlp_destroy(None)


def test_tune_table_round_trip_and_bounds():
    rc, w, d = R.rpca_tune_get(10, 200)
    assert rc == R.RPCA_OK and w >= 64 and d >= 1
    assert R.rpca_tune_set(10, 200, 4096, 2) == R.RPCA_OK
    assert R.rpca_tune_get(12, 250)[1:] == (4096, 2)      # same (k, n) bucket
    assert R.rpca_tune_get(10, 600)[1:] == (w, d)         # other bucket untouched
    assert R.rpca_tune_set(10, 200, w, d) == R.RPCA_OK
    assert R.rpca_tune_set(33, 200, 2048, 1) == R.RPCA_EINVAL
    assert R.rpca_tune_set(10, 200, 8, 1) == R.RPCA_EINVAL
    assert R.rpca_autotune(8, 10) == R.RPCA_EINVAL
    assert R.rpca_autotune(31, 10) == R.RPCA_EINVAL     # the k = 32 probes need 32 rows
    assert R.lib().rpca_sweep_layout(None, None) == R.RPCA_EINVAL


def test_batch_entry_points_reject_bad_arguments_before_hip():
    rc, b = R.rpca_batch_create([100, 50], [20, 10], [5, 11], [0.1, 0.1], [1.0, 1.0])   # k > n
    assert rc == R.RPCA_EINVAL and not b.value
    rc, b = R.rpca_batch_create([100], [20], [5], [0.0], [1.0])
    assert rc == R.RPCA_EINVAL
    assert R.rpca_batch_objgrad(None, [1], [1], [1], [1], [1], [1]) == R.RPCA_EINVAL
    rc, _ = R.rpca_batch_solve(None, [1], [1], [1])
    assert rc == R.RPCA_EINVAL
    assert R.rpca_batch_set_graphs(None, 1) == R.RPCA_EINVAL
    assert R.rpca_batch_instance_waves(None, 0)[0] == R.RPCA_EINVAL
    R.rpca_batch_destroy(None)


def test_frank_wolfe_entry_points_reject_bad_arguments_before_hip():
    for args in [(0, 10, 0.1, 1.0), (10, 0, 0.1, 1.0), (10, 10, 0.0, 1.0), (10, 10, 0.1, -1.0),
                 (10, 10, float("nan"), 1.0), ((1 << 31) + 1, 10, 0.1, 1.0), (10, (1 << 24) + 1, 0.1, 1.0)]:
        rc, h = R.rpca_fw_create(*args)
        assert rc == R.RPCA_EINVAL and not h.value
    assert R.rpca_fw_solve(None, 1, 1, 0.0, 10, 1e-6)[0] == R.RPCA_EINVAL
    assert R.rpca_fw_solve(None, 1, 1, 0.0, 10, 1e-6, -1.0)[0] == R.RPCA_EINVAL
    R.rpca_fw_destroy(None)


def test_frank_wolfe_info_layout_matches_header_order():
    text = open(R.HEADER_PATHS[-1]).read()
    body = re.search(r"typedef struct rpca_fw_info \{(.*?)\} rpca_fw_info;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    assert [f for f, _ in R.rpca_fw_info._fields_] == re.findall(r"(\w+)\s*;", body)


def test_frank_wolfe_profile_rejects_null():
    assert R.lib().rpca_fw_profile_enable(None, 1) == R.RPCA_EINVAL
    assert R.rpca_fw_profile_read(None)[0] == R.RPCA_EINVAL


def test_set_elastic_rejects_bad_arguments():
    L = R.lib()
    assert L.rpca_set_elastic(None, 0.5) == R.RPCA_EINVAL


def test_prox_solve_rejects_bad_arguments_before_hip():
    assert R.rpca_prox_solve(None, 1, 1, 1)[0] == R.RPCA_EINVAL
    L = R.lib()
    info = R.rpca_prox_info()
    import ctypes as C
    for args in [(0, 1e-8, 10, 1), (10, -1.0, 10, 1), (10, 1e-8, 33, 1), (10, 1e-8, 10, 9)]:
        assert L.rpca_prox_solve(C.c_void_p(1), 1, 1, 1, *args, 7, C.byref(info), None) == R.RPCA_EINVAL


def test_prox_info_layout_matches_header_order():
    text = open(R.HEADER_PATH).read()
    body = re.search(r"typedef struct rpca_prox_info \{(.*?)\} rpca_prox_info;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    assert [f for f, _ in R.rpca_prox_info._fields_] == re.findall(r"(\w+)\s*;", body)


def test_objgrad_noalloc_rejects_bad_arguments_and_oversize_before_hip():
    d = ctypes.c_void_p(16)
    call = R.lib().rpca_objgrad_noalloc
    assert call(100, 50, 0, 0.1, 1.0, None, d, d, d, d, d, d, None) == R.RPCA_EINVAL
    assert call(100, 50, 33, 0.1, 1.0, None, d, d, d, d, d, d, None) == R.RPCA_EINVAL
    assert call(10, 50, 11, 0.1, 1.0, None, d, d, d, d, d, d, None) == R.RPCA_EINVAL
    assert call(100, 50, 5, 0.0, 1.0, None, d, d, d, d, d, d, None) == R.RPCA_EINVAL
    assert call(100, 50, 5, 0.1, float("inf"), None, d, d, d, d, d, d, None) == R.RPCA_EINVAL
    assert call(100, 50, 5, 0.1, 1.0, None, None, d, d, d, d, d, None) == R.RPCA_EINVAL
    assert call(100, 50, 5, 0.1, 1.0, None, d, d, d, d, d, None, None) == R.RPCA_EINVAL
    # many column chunks of a tall matrix: the G V partials exceed the fixed array
    assert call(1 << 22, 1 << 14, 32, 0.1, 1.0, None, d, d, d, d, d, d, None) == R.RPCA_ETOOBIG


def test_set_graphs_rejects_null_context():
    assert R.lib().rpca_set_graphs(None, 1) == R.RPCA_EINVAL


def test_create_device_mask_rejects_null_mask():
    rc, _ = R.rpca_create_device_mask(64, 32, 4, 0.1, 1.0, None, 0)
    assert rc == R.RPCA_EINVAL
    rc, _ = R.rpca_create_device_mask(64, 32, 4, 0.1, 1.0, 16, -1)
    assert rc == R.RPCA_EINVAL
