"""GPU: sweep 1 in pull form (Section 5, Algorithms 5-6) against the oracle.

The pull engine sums, for every output y, p(x) emb(y,x) over the supersequences x
of y enumerated by Algorithm 6 (with the tail read as y's last symbol), without
atomics.  Its r, D and bounds must match the oracle (FP64 within 1e-12 relative /
1e-10 bits), the other engines, and be bitwise reproducible.
"""
import math

import numpy as np
import pytest
import torch

import bdc_inputs as inp
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


@pytest.mark.parametrize("n", [1, 2, 3, 6, 9, 12])
def test_pull_eval_matches_oracle(ba, n):
    d = 0.55
    lp = inp.random_logp(n, seed=80 + n, spread=2.0)
    W = bdc.channel_dense(n, d)
    ev = bdc.evaluate(W, lp)
    c = ba.Context(n, d, engine=ba.ENGINE_PULL)
    got = c.eval(torch.from_numpy(lp))
    c.close()
    r_o = np.exp(bdc.normalise_logp(lp)) @ bdc.emb_dense(n)
    # the GPU keeps r scaled by e^{-M}, M = max log p (returned as "M")
    r = got["r"].cpu().numpy() * math.exp(got["M"])
    assert np.allclose(r, r_o, rtol=1e-12, atol=0)
    assert abs(got["L"] - ev.L / LN2) < 1e-10 and abs(got["U"] - ev.U / LN2) < 1e-10
    assert np.max(np.abs(got["D"].cpu().numpy() - ev.D)) < 1e-10


def test_pull_agrees_with_other_engines_and_is_deterministic(ba):
    n, d = 14, 0.7
    lp = inp.random_logp(n, seed=91, spread=2.0)
    out = {}
    for name, eng in (("pull", ba.ENGINE_PULL), ("stream", ba.ENGINE_STREAM), ("factored", ba.ENGINE_FACTORED)):
        c = ba.Context(n, d, engine=eng)
        a = c.eval(torch.from_numpy(lp))
        out[name] = (a["r"].cpu().numpy(), a["L"], a["U"])
        if name == "pull":
            b = c.eval(torch.from_numpy(lp))
            assert np.array_equal(a["r"].cpu().numpy(), b["r"].cpu().numpy())
        c.close()
    for other in ("stream", "factored"):
        assert np.allclose(out["pull"][0], out[other][0], rtol=1e-12, atol=0)
        assert abs(out["pull"][1] - out[other][1]) < 1e-11 and abs(out["pull"][2] - out[other][2]) < 1e-11


def test_pull_fp64_iterates_match_oracle(ba):
    n, d, iters = 8, 0.5, 20
    W = bdc.channel_dense(n, d)
    lp_o = bdc.ba_iterate(W, bdc.uniform_logp(n), iters)
    c = ba.Context(n, d, engine=ba.ENGINE_PULL)
    c.step(iters)
    lp = c.get_logp().cpu().numpy()
    c.close()
    assert np.max(np.abs(lp - lp_o)) < 1e-10


def test_pull_fp32_batch_matches_factored(ba):
    ns, ds = [10, 12, 10], [0.64, 0.8, 0.96]
    out = []
    for eng in (ba.ENGINE_PULL, ba.ENGINE_FACTORED):
        c = ba.Context(ns, ds, prec=ba.PREC_FP32_LOG, engine=eng)
        c.step(20)
        out.append((c.get_logp().cpu().numpy(), c.bounds()))
        c.close()
    assert np.max(np.abs(out[0][0] - out[1][0])) < 1e-3
    for a, b in zip(out[0][1], out[1][1]):
        assert np.max(np.abs(np.array(a) - np.array(b))) < 1e-6
