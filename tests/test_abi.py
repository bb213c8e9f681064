"""The C ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host before touching a device (no compute without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfsft.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bfsft_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_0801_1524_amd as bf
    if not os.path.exists(bf.LIB_PATH):
        from paper_0801_1524_amd import build
        build.build()
    return bf.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("bfsft_plan_create", "bfsft_execute", "bfsft_execute_adjoint", "bfsft_destroy", "bfsft_strerror",
                 "bfsft_plan_info", "bfsft_plan_create_batched", "bfsft_execute_batched"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_destroy_null(lib):
    for s in (0, -1, -2, -3, -4):
        assert lib.bfsft_strerror(s)
    lib.bfsft_destroy(None)  # NULL is a no-op


@pytest.mark.parametrize("d,N,p,prec", [
    (1, 256, 5, 0),      # d not 2 or 3
    (4, 256, 5, 0),
    (2, 256, 2, 0),      # p = 2: singular matching system
    (2, 256, 13, 0),     # p beyond the 2D tile bound
    (3, 256, 9, 0),      # p beyond the 3D tile bound
    (3, 256, 8, 0),      # 3D p = 8 at FP64: one box and its children exceed the LDS
    (2, 1, 5, 0),        # N < 2
    (2, 256, 5, 7),      # unknown precision
    (2, 256, 5, 5),
    (2, 256, 5, -1),
    (3, 256, 5, 2),      # the split contraction formats are 2D only
    (3, 256, 5, 3),
])
def test_invalid_scalars_rejected_on_host(lib, d, N, p, prec):
    h = ctypes.c_void_p(1234)
    rc = lib.bfsft_plan_create(ctypes.byref(h), d, N, p, prec, None, 0, None, 0, None)
    assert rc == -1
    assert h.value is None
    assert lib.bfsft_last_error()


def test_negative_count_and_null_points_rejected(lib):
    h = ctypes.c_void_p()
    assert lib.bfsft_plan_create(ctypes.byref(h), 2, 256, 5, 0, None, -1, None, 0, None) == -1
    assert lib.bfsft_plan_create(ctypes.byref(h), 2, 256, 5, 0, None, 10, None, 0, None) == -1
    assert lib.bfsft_plan_create(None, 2, 256, 5, 0, None, 0, None, 0, None) == -1


def test_execute_null_plan(lib):
    assert lib.bfsft_execute(None, None, None) == -1
    assert lib.bfsft_execute_batched(None, None, None) == -1


def test_batched_without_problems_rejected(lib):
    h = ctypes.c_void_p(1234)
    assert lib.bfsft_plan_create_batched(ctypes.byref(h), 0, None, 2, 5, 0, None) == -1
    assert h.value is None
    assert lib.bfsft_plan_create_batched(ctypes.byref(h), 3, None, 2, 5, 0, None) == -1
    assert lib.bfsft_last_error()
    assert lib.bfsft_execute_adjoint(None, None, None) == -1


def test_precision_values_match_the_boundary():
    """The precision codes of the header: FP64 = 0, FP32 = 1, FP16X2 = 2,
    BF16X3 = 3, MIXED = 4; the binding uses the same values."""
    import paper_0801_1524_amd as bf
    text = open(HEADER).read()
    vals = dict(re.findall(r"#define (BFSFT_(?:FP64|FP32|FP16X2|BF16X3|MIXED))\s+(\d+)", text))
    assert vals == {"BFSFT_FP64": "0", "BFSFT_FP32": "1", "BFSFT_FP16X2": "2", "BFSFT_BF16X3": "3",
                    "BFSFT_MIXED": "4"}
    for name, code in bf.PRECISIONS.items():
        assert vals["BFSFT_" + name.upper()] == str(code)


def test_measurement_helpers_reject_bad_arguments(lib):
    # both helpers check their arguments before any device call
    out = ctypes.c_double()
    assert lib.bfsft_mfma_f64_rate(0, 10, None, ctypes.byref(out)) == -1
    assert lib.bfsft_mfma_f64_rate(2, 0, None, ctypes.byref(out)) == -1
    assert lib.bfsft_mfma_f64_rate(2, 10, None, None) == -1
    assert lib.bfsft_copy_rate(3, 1 << 20, 1, None, ctypes.byref(out)) == -1
    assert lib.bfsft_copy_rate(8, 1 << 10, 1, None, ctypes.byref(out)) == -1
    assert lib.bfsft_last_error()
