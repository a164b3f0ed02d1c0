"""ba_bind_static: the entry point for callers that cannot allocate device memory.

A context bound to the library's static per-GPU array must give exactly what the
same context bound to a caller workspace (ba_bind) gives: same kernels, same
order, and a deterministic init pass, so iterates and certified bounds are
bitwise equal.  Two binds in a row, the second with a smaller instance set; the
context bound first loses the array; a context too large for it is refused.
"""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ba():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05867_amd as m
    m.lib()
    return m


def say(*a):
    print(*a, flush=True)


def new_ctx(L, ns, ds, prec):
    h = ctypes.c_void_p()
    n = (ctypes.c_int * len(ns))(*ns)
    d = (ctypes.c_double * len(ds))(*ds)
    assert L.ba_init_batch(len(ns), n, d, prec, 25, ctypes.byref(h)) == 0
    return h


def outcome(L, h, ns):
    count = len(ns)
    lo = (ctypes.c_double * count)()
    hi = (ctypes.c_double * count)()
    assert L.ba_bounds(h, lo, hi) == 0, L.ba_last_error(h)
    lp = torch.empty(sum(1 << n for n in ns), dtype=torch.float64, device="cuda:0")
    assert L.ba_get_logp(h, ctypes.c_void_p(lp.data_ptr())) == 0
    torch.cuda.synchronize()
    return list(lo), list(hi), lp.cpu().numpy()


def test_bind_static_equals_bind(ba):
    L = ba.lib()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    cases = [([14, 12, 14], [0.64, 0.8, 0.95], ba.PREC_FP32_LOG, 60),
             ([10], [0.7], ba.PREC_FP64, 40)]
    prev = None
    for ns, ds, prec, steps in cases:
        say("bind_static: n=%s d=%s prec=%d steps=%d" % (ns, ds, prec, steps))
        h = new_ctx(L, ns, ds, prec)
        assert L.ba_bind_static(h, sp) == 0, L.ba_last_error(h)
        ref = ba.Context(ns, ds, prec=prec, cert_every=25, stream=stream)
        if prev is not None:
            # binding this context took the array from the previous one
            assert L.ba_step(prev, 1) == ba.BA_ESTATE
            assert b"static workspace" in L.ba_last_error(prev)
            L.ba_free(prev)
        assert L.ba_step(h, steps) == 0
        ref.step(steps)
        got = outcome(L, h, ns)
        lo, hi = ref.bounds()
        want_lp = ref.get_logp().cpu().numpy()
        assert got[0] == lo and got[1] == hi
        assert np.array_equal(got[2], want_lp)
        # a stopping-rule run continues on both in the same way
        done = ctypes.c_int()
        assert L.ba_run(h, ctypes.c_double(1e-12), 50, ctypes.byref(done)) == 0
        assert ref.run(1e-12, 50) == done.value
        got = outcome(L, h, ns)
        lo, hi = ref.bounds()
        assert got[0] == lo and got[1] == hi
        assert np.array_equal(got[2], ref.get_logp().cpu().numpy())
        ref.close()
        prev = h
    # too large for the static array: refused with the sizes, nothing bound
    big = new_ctx(L, [20], [0.8], ba.PREC_FP32_LOG)
    assert L.ba_bind_static(big, sp) == ba.BA_ENOMEM
    assert b"static workspace" in L.ba_last_error(big)
    assert L.ba_step(big, 1) == ba.BA_ESTATE
    L.ba_free(big)
    # the last static context still owns the array and works
    assert L.ba_step(prev, 1) == 0
    L.ba_free(prev)
