"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, fills defaults, and rejects bad arguments before any HIP call
(so these run without a GPU)."""
import ctypes
import re

import pytest

from paper_1702_02241_amd import rpca as R


def _declared_symbols():
    text = open(R.HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rpca_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = R.lib()
    names = _declared_symbols()
    assert "rpca_create" in names and "rpca_solve" in names and "rpca_certificate" in names
    for name in names:
        assert hasattr(L, name), f"{name} declared in rpca.h but not exported"


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


def test_null_context_rejected():
    assert R.rpca_objgrad(None, 1, 1, 1, 1, 1, 1, 0) == R.RPCA_EINVAL
    rc, _ = R.rpca_solve(None, 1, 1, 1)
    assert rc == R.RPCA_EINVAL
    rc, _ = R.rpca_certificate(None, 1, 1, 1)
    assert rc == R.RPCA_EINVAL
    R.rpca_destroy(None)


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
