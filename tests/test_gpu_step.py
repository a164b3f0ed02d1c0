"""GPU: the update step eta (entropic mirror ascent on the iterate; eta = 1 is BA).

With eta != 1 the iteration is p <- p e^{eta D} / Z; the oracle's mirror ascent
(theta <- theta + eta D, p = softmax theta) is the same map.  The bounds reported
for any iterate stay valid, so every run must bracket the oracle's capacity.
"""
import math

import numpy as np
import pytest
import torch

from oracle import bdc

pytestmark = pytest.mark.gpu
LN2 = math.log(2.0)


@pytest.fixture(scope="module")
def ba():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05867_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("engine", ["factored", "stream"])
@pytest.mark.parametrize("eta", [0.5, 1.7, 2.5])
def test_step_matches_oracle_mirror_ascent(ba, engine, eta):
    n, d, steps = 8, 0.6, 15
    eng = ba.ENGINE_FACTORED if engine == "factored" else ba.ENGINE_STREAM
    th = bdc.mirror_ascent(n, d, np.zeros(1 << n), eta, steps)
    lp_o = bdc.normalise_logp(th)
    W = bdc.channel_dense(n, d)
    L_o, U_o = bdc.certify(W, lp_o)
    c = ba.Context(n, d, engine=eng)
    c.set_step(eta)
    c.step(steps)
    lp = c.get_logp().cpu().numpy()
    lo, hi = c.bounds()
    c.close()
    assert np.max(np.abs(lp - lp_o)) < 1e-10
    assert abs(lo[0] - L_o) < 1e-10 and abs(hi[0] - U_o) < 1e-10


def test_step_one_is_ba(ba):
    """eta = 1 set explicitly gives bitwise the default iteration."""
    out = []
    for set_it in (False, True):
        c = ba.Context([10, 12], [0.7, 0.9], prec=ba.PREC_FP32_LOG)
        if set_it:
            c.set_step(1.0)
        c.step(30)
        out.append(c.get_logp().cpu().numpy())
        c.close()
    assert np.array_equal(out[0], out[1])


def test_step_symmetric_mode(ba):
    """The symmetric kernels with a step equal the full kernels with the same step."""
    out = []
    for sym in (False, True):
        c = ba.Context(12, 0.75)
        c.set_step(2.0)
        if sym:
            c.set_symmetry(True)
        c.step(20)
        out.append((c.get_logp().cpu().numpy(), c.bounds()))
        c.close()
    assert np.max(np.abs(out[0][0] - out[1][0])) < 1e-12
    assert abs(out[0][1][0][0] - out[1][1][0][0]) < 1e-12 and abs(out[0][1][1][0] - out[1][1][1][0]) < 1e-12


def test_step_fp32_run_brackets_capacity(ba, oracle_native):
    """FP32 iterates with eta = 2, certified in FP64: the best bracket contains the
    oracle's FP64 bracket's overlap (bounds are valid for any iterate)."""
    n, d = 10, 0.8
    csr = oracle_native.CSR(n)
    lp = bdc.uniform_logp(n)
    for _ in range(3000):
        D, L, U, I, _ = csr.evaluate(d, lp, floor_nats=700.0)
        lp = bdc.floor_logp(bdc.normalise_logp(lp) + D - L, 700.0)
    D, L, U, I, _ = csr.evaluate(d, lp, floor_nats=700.0)
    L_o, U_o = L / LN2, U / LN2
    c = ba.Context(n, d, prec=ba.PREC_FP32_LOG, cert_every=50)
    c.set_step(2.0)
    c.set_stop_rule(ba.STOP_BEST)
    c.run(1e-6, 20000)
    lo, hi, its = c.best_bounds()
    c.close()
    print("eta=2: iters=%d gap=%.3e" % (its[0], hi[0] - lo[0]), flush=True)
    assert lo[0] <= U_o + 1e-12 and L_o <= hi[0] + 1e-12
    assert hi[0] - lo[0] < 1e-4


def test_step_rejects_bad_values(ba):
    c = ba.Context(6, 0.5)
    for bad in (0.0, -1.0, 9.0, float("nan")):
        with pytest.raises(ba.BAError) as e:
            c.set_step(bad)
        assert e.value.code == ba.BA_EINVAL
    c.close()


@pytest.mark.parametrize("floor", [50.0, 80.0])
def test_iterate_floor_matches_oracle(ba, floor):
    """ba_set_floor: FP64 iterates floored at `floor` nats below their maximum equal
    the oracle's floored BA iterates (ba_update with floor_nats) within 1e-9 nats
    after 1500 iterations of n = 8, d = 0.8, where ~90 inputs sit at the floor; the
    certified bounds of that iterate match the oracle's certification."""
    n, d = 8, 0.8
    W = bdc.channel_dense(n, d)
    ctx = ba.Context(n, d, prec=ba.PREC_FP64)
    ctx.set_floor(floor)
    ctx.step(1500)
    got = bdc.normalise_logp(ctx.get_logp().cpu().numpy())
    want = bdc.ba_iterate(W, bdc.uniform_logp(n), 1500, floor_nats=floor)
    assert int(np.sum(want <= want.max() - floor + 1e-9)) > 10
    assert np.max(np.abs(got - want)) < 1e-9
    lo, hi = ctx.bounds()
    L, U = bdc.certify(W, want)
    assert abs(lo[0] - L) < 1e-10 and abs(hi[0] - U) < 1e-10
    ctx.close()
