"""The C-ABI library loads, exports every entry point of include/ba.h and
rejects bad arguments on the host (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ba.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ba_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2604_05867_amd as ba
    if not os.path.exists(ba.LIB_PATH):
        pytest.skip("libba.so not built")
    return ba.lib()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for want in ["ba_init", "ba_init_batch", "ba_bind", "ba_step", "ba_run", "ba_bounds", "ba_grad",
                 "ba_eval", "ba_get_logp", "ba_set_logp", "ba_row_counts", "ba_verify_counts", "ba_free",
                 "ba_strerror", "ba_workspace_bytes", "ba_time_kernels"]:
        assert want in syms


def test_library_exports_every_declared_symbol(L):
    for s in declared_symbols():
        assert hasattr(L, s), s


def test_argument_errors(L):
    h = ctypes.c_void_p()
    assert L.ba_init(0, 0.5, ctypes.byref(h)) == -1
    assert L.ba_init(21, 0.5, ctypes.byref(h)) == -1
    assert L.ba_init(5, -0.1, ctypes.byref(h)) == -1
    assert L.ba_init(5, 1.1, ctypes.byref(h)) == -1
    assert L.ba_init(5, float("nan"), ctypes.byref(h)) == -1
    n = (ctypes.c_int * 2)(5, 6)
    d = (ctypes.c_double * 2)(0.5, 0.5)
    assert L.ba_init_batch(2, n, d, 7, 50, ctypes.byref(h)) == -1  # bad precision
    assert L.ba_init_batch(2, n, d, 0, 0, ctypes.byref(h)) == -1   # cert_every < 1
    assert L.ba_init_batch(0, n, d, 0, 1, ctypes.byref(h)) == -1
    assert L.ba_init(5, 0.5, ctypes.byref(h)) == 0
    # every compute call before bind is a state error, nothing crashes
    assert L.ba_step(h, 1) == -4
    lo = ctypes.c_double()
    hi = ctypes.c_double()
    assert L.ba_bounds(h, ctypes.byref(lo), ctypes.byref(hi)) == -4
    assert b"ba_bind" in L.ba_last_error(h)
    assert L.ba_set_engine(h, 5) == -1
    assert L.ba_set_engine(h, 0) == 0
    # iterate floor: 50..700 nats for FP64 iterates
    for bad in (0.0, 49.9, 701.0, float("nan"), float("inf")):
        assert L.ba_set_floor(h, ctypes.c_double(bad)) == -1
    assert L.ba_set_floor(h, ctypes.c_double(80.0)) == 0
    assert L.ba_set_floor(h, ctypes.c_double(700.0)) == 0
    sz = ctypes.c_size_t()
    assert L.ba_workspace_bytes(h, ctypes.byref(sz)) == 0 and sz.value > 0
    assert L.ba_bind(h, None, sz.value, None) == -1
    assert L.ba_bind(h, ctypes.c_void_p(256), 16, None) == -2  # too small, checked before any device use
    L.ba_free(h)
    h32 = ctypes.c_void_p()
    assert L.ba_init_batch(2, n, d, 1, 50, ctypes.byref(h32)) == 0
    assert L.ba_set_floor(h32, ctypes.c_double(88.0)) == -1   # e^-88 is below the normal floats
    assert L.ba_set_floor(h32, ctypes.c_double(87.0)) == 0
    L.ba_free(h32)
    L.ba_free(None)
    assert L.ba_strerror(-5) == b"non-finite value"


def test_nnz_formula(L):
    for n in range(0, 21):
        assert L.ba_nnz(n) == 2 * 3 ** n - 2 ** n
