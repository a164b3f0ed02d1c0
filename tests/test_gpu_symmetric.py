"""GPU: complement-symmetric iteration (Appendix A, Theorem 4).

From the uniform law every BA iterate satisfies p(cpl x) = p(x), so the factored
products can be evaluated on the canonical half.  The symmetric mode must give the
iterates and bounds of the full kernels (FP64: within 1e-12; FP32: same rounding
class) and of the oracle's BA, and refuse laws that are not complement-symmetric.
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


def say(*a):
    print(*a, flush=True)


def run_pair(ba, ns, ds, prec, iters, exact_k=None, fuse=None):
    """(logp, bounds) after `iters` iterations with the full and the symmetric kernels."""
    out = []
    for sym in (False, True):
        if exact_k is not None:
            c = ba.Context(ns, None, prec=prec, k=exact_k)
        else:
            c = ba.Context(ns, ds, prec=prec)
        if fuse is not None:
            c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        if sym:
            c.set_symmetry(True)
        c.step(iters)
        lo, hi = c.bounds()
        out.append((c.get_logp().cpu().numpy(), np.array(lo), np.array(hi)))
        c.close()
    return out


@pytest.mark.parametrize("fuse", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [4, 6, 8, 10, 12, 14, 16])
def test_symmetric_fp64_equals_full(ba, n, fuse):
    say("symmetric fp64 n=%d fuse=%d" % (n, fuse))
    (lp_f, lo_f, hi_f), (lp_s, lo_s, hi_s) = run_pair(ba, n, 0.7, ba.PREC_FP64, 30, fuse=fuse)
    assert np.max(np.abs(lp_f - lp_s)) < 1e-12
    assert np.max(np.abs(lo_f - lo_s)) < 1e-12 and np.max(np.abs(hi_f - hi_s)) < 1e-12
    # the symmetric iterate is exactly invariant under complement
    assert np.array_equal(lp_s, lp_s[::-1])


def test_full_kernels_keep_complement_symmetry_bitwise(ba):
    """Theorem 4 on the full kernels of the n = 20 FP32 plan (first eight positions,
    twelve-position launches, fused D launch): from the uniform law every iterate is
    complement-invariant, and these kernels keep it bit for bit (the sum at (cpl y,
    cpl s) adds the same terms as at (y, s), two operands swapped), over 7 iterations in
    one call and 3 more in another.  (The four- and eight-position kernels of the other
    plans group some sums differently at mirrored positions, so there the invariance
    holds to rounding.)"""
    n = 20
    say("full kernels complement symmetry n=20 fp32")
    ns, ds = [n] * 3, [0.64, 0.8, 0.95]
    c = ba.Context(ns, ds, prec=ba.PREC_FP32_LOG)
    c.step(7)
    c.step(3)
    lp = c.get_logp().cpu().numpy().reshape(len(ns), 1 << n)
    c.close()
    for k in range(len(ns)):
        assert np.array_equal(lp[k], lp[k][::-1])


@pytest.mark.parametrize("n", [8, 14])
def test_symmetric_fp64_matches_oracle(ba, n):
    """Against the oracle's dense or sparse BA from the uniform law (Section 2.3)."""
    d, iters = 0.6, 12
    if n <= 8:
        W = bdc.channel_dense(n, d)
        lp_o = bdc.ba_iterate(W, bdc.uniform_logp(n), iters)
        L_o, U_o = bdc.certify(W, lp_o)
    else:
        import oracle.native as on
        csr = on.CSR(n)
        lp_o = bdc.uniform_logp(n)
        for _ in range(iters):
            D, L, U, I, _ = csr.evaluate(d, lp_o, floor_nats=700.0)
            lp_o = bdc.floor_logp(bdc.normalise_logp(lp_o) + D - L, 700.0)
        _, L, U, _, _ = csr.evaluate(d, lp_o, floor_nats=700.0)
        L_o, U_o = L / LN2, U / LN2
    c = ba.Context(n, d)
    c.set_symmetry(True)
    c.step(iters)
    lp = c.get_logp().cpu().numpy()
    lo, hi = c.bounds()
    c.close()
    assert np.max(np.abs(lp - lp_o)) < 1e-10
    assert abs(lo[0] - L_o) < 1e-10 and abs(hi[0] - U_o) < 1e-10


def test_symmetric_fp32_batch_mixed_n(ba):
    """A batch with odd n (full kernels) and even n (symmetric kernels), FP32
    iterates: same iterates as the full kernels up to FP32 rounding, certified
    bounds within 1e-6 bits."""
    ns = [7, 8, 10, 12, 10]
    ds = [0.64, 0.7, 0.8, 0.9, 0.96]
    (lp_f, lo_f, hi_f), (lp_s, lo_s, hi_s) = run_pair(ba, ns, ds, ba.PREC_FP32_LOG, 200)
    assert np.max(np.abs(lp_f - lp_s)) < 1e-2
    assert np.max(np.abs(lo_f - lo_s)) < 1e-6 and np.max(np.abs(hi_f - hi_s)) < 1e-6


def test_symmetric_exact_channel(ba):
    """Exact channels BDC_{n,k} are complement-invariant too (Section 2.2)."""
    (lp_f, lo_f, hi_f), (lp_s, lo_s, hi_s) = run_pair(ba, [10, 12], None, ba.PREC_FP64, 25, exact_k=[5, 4])
    assert np.max(np.abs(lp_f - lp_s)) < 1e-12
    assert np.max(np.abs(lo_f - lo_s)) < 1e-12 and np.max(np.abs(hi_f - hi_s)) < 1e-12


@pytest.mark.parametrize("fuse", [4, 8])
def test_symmetric_n20_fp32(ba, fuse):
    """The benchmark shape: n = 20, three instances, FP32 iterates, with the
    complement-symmetric kernels (launch plan 4) or the full plan on half the rows and
    column tiles (plan 8).  The two sets sum in different orders (or group the records
    differently) and the full set forms its D records in single precision, so the FP32
    iterates agree to rounding (log p of magnitude ~14 has an ulp of ~1e-6) and their
    FP64-certified bounds within 1e-6 bits."""
    say("symmetric n=20 fp32 fuse=%d" % fuse)
    ds = [0.64, 0.8, 0.95]
    (lp_f, lo_f, hi_f), (lp_s, lo_s, hi_s) = run_pair(ba, [20] * 3, ds, ba.PREC_FP32_LOG, 6, fuse=fuse)
    assert np.max(np.abs(lp_f - lp_s)) < 1e-4
    assert np.max(np.abs(lo_f - lo_s)) < 1e-6 and np.max(np.abs(hi_f - hi_s)) < 1e-6
    X = 1 << 20
    for b in range(3):
        seg = lp_s[b * X:(b + 1) * X]
        assert np.array_equal(seg, seg[::-1])


@pytest.mark.parametrize("per_call", [1, 2, 3, 7])
def test_half_plan_n20_fp32_calls(ba, per_call):
    """The half plan (complement-symmetric iterate, n = 20, FP32, plan 8: the full
    plan's kernels on the rows that start with 0 and the column tiles whose first bit
    is 0) against the full plan from the uniform law, 7 iterations in calls of 1, 2, 3
    or 7: log p within 4e-5 and the certified bounds within 1e-6 bits (the D records
    count each input of a pair twice, so L rounds differently); the half iterate is
    exactly complement-invariant; with 7 per call the same launches ran (9 forward, 14
    backward, one record reduction)."""
    say("half plan n=20 per_call=%d" % per_call)
    ds = [0.64, 0.8, 0.95]
    out = []
    for sym in (False, True):
        c = ba.Context([20] * 3, ds, prec=ba.PREC_FP32_LOG)
        if sym:
            c.set_symmetry(True)
        done = 0
        while done < 7:
            k = min(per_call, 7 - done)
            c.step(k)
            done += k
        lo, hi = c.bounds()
        out.append((c.get_logp().cpu().numpy(), np.array(lo), np.array(hi)))
        if per_call == 7 and sym:
            c.set_logp(torch.full((3 << 20,), -20 * LN2, dtype=torch.float64))
            t = c.time_kernels(7)
            assert t["sweep1"][1] == 9 and t["sweep2"][1] == 14 and t["reduce"][1] == 1
        c.close()
    (lp_f, lo_f, hi_f), (lp_s, lo_s, hi_s) = out
    assert np.max(np.abs(lp_f - lp_s)) < 4e-5
    assert np.max(np.abs(lo_f - lo_s)) < 1e-6 and np.max(np.abs(hi_f - hi_s)) < 1e-6
    X = 1 << 20
    for b in range(3):
        seg = lp_s[b * X:(b + 1) * X]
        assert np.array_equal(seg, seg[::-1])


@pytest.mark.parametrize("fuse", [2, 4])
def test_symmetric_n20_fp64(ba, fuse):
    """n = 20 in FP64 (8 roots per eight-position block), where the symmetric
    backward sweep takes its first eight positions in one launch from the compact v
    and the forward sweep its last four in one launch: iterates and bounds equal
    those of the full kernels."""
    say("symmetric fp64 n=20 fuse=%d" % fuse)
    (lp_f, lo_f, hi_f), (lp_s, lo_s, hi_s) = run_pair(ba, 20, 0.8, ba.PREC_FP64, 3, fuse=fuse)
    assert np.max(np.abs(lp_f - lp_s)) < 1e-12
    assert np.max(np.abs(lo_f - lo_s)) < 1e-12 and np.max(np.abs(hi_f - hi_s)) < 1e-12
    assert np.array_equal(lp_s, lp_s[::-1])


def test_symmetric_rejects_asymmetric_law(ba):
    n = 10
    c = ba.Context(n, 0.7)
    lp = inp.random_logp(n, seed=5, spread=2.0)
    c.set_logp(torch.from_numpy(lp))
    with pytest.raises(ba.BAError) as e:
        c.set_symmetry(True)
    assert e.value.code == ba.BA_EINVAL
    # a complement-symmetric law is accepted and iterates like the full kernels
    sym = 0.5 * (lp + lp[::-1])
    c.set_logp(torch.from_numpy(np.ascontiguousarray(sym)))
    c.set_symmetry(True)
    c.step(10)
    lp_s = c.get_logp().cpu().numpy()
    # setting an asymmetric law while the mode is on switches it off with an error
    with pytest.raises(ba.BAError):
        c.set_logp(torch.from_numpy(lp))
    c.close()
    f = ba.Context(n, 0.7)
    f.set_logp(torch.from_numpy(np.ascontiguousarray(sym)))
    f.step(10)
    assert np.max(np.abs(f.get_logp().cpu().numpy() - lp_s)) < 1e-12
    f.close()


def test_symmetric_graph_replay(ba):
    """ba_run's captured graph with the symmetric kernels equals eager launches."""
    s = torch.cuda.Stream()
    c = ba.Context([8, 10], [0.6, 0.9], prec=ba.PREC_FP32_LOG, cert_every=20, stream=s)
    c.set_symmetry(True)
    start = torch.zeros((1 << 8) + (1 << 10), dtype=torch.float64)
    out = []
    for graphs in (False, True):
        c.set_graphs(graphs)
        with torch.cuda.stream(s):
            c.set_logp(start)
            done = c.run(1e-7, 300)
            lo, hi, its = c.best_bounds()
            lp = c.get_logp().cpu().numpy()
        s.synchronize()
        out.append((done, lo, hi, its, lp))
    c.close()
    assert out[0][0] == out[1][0] and out[0][3] == out[1][3]
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]
    assert np.array_equal(out[0][4], out[1][4])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_symmetric_fused_update_is_bitwise_separate(ba, prec):
    """Within one step call the symmetric kernels make the update of each iteration
    but the last inside the next iteration's first forward launch; the iterates and
    bounds equal those of one-iteration calls (separate update launches) bit for
    bit, with and without a step eta.  (Plan 4: at n = 20 with FP32 iterates plan 8
    runs the half plan instead, whose in-call updates shift by a max and are tested
    against the full plan to rounding.)"""
    p = ba.PREC_FP64 if prec == "fp64" else ba.PREC_FP32_LOG
    ns, ds = ([12, 14], [0.6, 0.9]) if prec == "fp64" else ([16, 20], [0.7, 0.95])
    say("symmetric fused update", prec)
    # one context, reset between runs
    c = ba.Context(ns, ds, prec=p)
    c.set_tuning(ba.TUNE_FACTORED_FUSE, 4)
    c.set_symmetry(True)
    start = torch.tensor(np.concatenate([np.full(1 << m, -m * LN2) for m in ns]))
    for eta in (1.0, 1.8):
        out = []
        for per_call in (1, 7):
            c.set_logp(start)
            c.set_step(eta)
            for _ in range(7 // per_call):
                c.step(per_call)
            out.append((c.get_logp().cpu().numpy(), c.bounds()))
        assert np.array_equal(out[0][0], out[1][0])
        assert out[0][1] == out[1][1]
        lp = out[1][0]
        off = 0
        for m in ns:  # still exactly complement-invariant
            assert np.array_equal(lp[off:off + (1 << m)], lp[off:off + (1 << m)][::-1])
            off += 1 << m
    c.close()


# ---------------------------------------------------------------------------
# Algorithm 7: the stream engine's output law over complement/reversal orbits
# ---------------------------------------------------------------------------

def stream_pair(ba, ns, ds, prec, iters):
    """(logp, bounds) after `iters` stream-engine iterations with the full scatter
    and with Algorithm 7 (ba_set_symmetry(2))."""
    out = []
    for mode in (0, 2):
        c = ba.Context(ns, ds, prec=prec, engine=ba.ENGINE_STREAM)
        if mode:
            c.set_symmetry(mode)
        c.step(iters)
        lo, hi = c.bounds()
        out.append((c.get_logp().cpu().numpy(), np.array(lo), np.array(hi)))
        c.close()
    return out


@pytest.mark.parametrize("n", [5, 8, 10])
def test_orbit_scatter_matches_oracle(ba, n):
    """Algorithm 7 (representative inputs, weights |O_x| / |O_y|, outputs filled from
    their orbit's representative) inside the stream engine's iterations: FP64
    iterates and certified bounds within 1e-10 of the oracle's BA from the uniform
    law; the oracle's own Algorithm 7 reproduces the output law of the iterate."""
    d = 0.7
    W = bdc.channel_dense(n, d)
    c = ba.Context(n, d, prec=ba.PREC_FP64, engine=ba.ENGINE_STREAM)
    c.set_symmetry(2)
    c.step(20)
    lp = c.get_logp().cpu().numpy()
    want = bdc.ba_iterate(W, bdc.uniform_logp(n), 20)
    assert np.max(np.abs(lp - want)) < 1e-10
    lo, hi = c.bounds()
    L, U = bdc.certify(W, want)
    assert abs(lo[0] - L) < 1e-10 and abs(hi[0] - U) < 1e-10
    E = bdc.emb_dense(n)
    assert np.allclose(bdc.r_orbits(n, lp), np.exp(bdc.normalise_logp(lp)) @ E, rtol=1e-12, atol=0)
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_orbit_scatter_equals_full_scatter(ba, prec):
    """Batches with odd and even n (orbits of size 1, 2 and 4 at every length): the
    Algorithm 7 scatter gives the iterates and bounds of the full scatter (FP64
    within 1e-12; FP32 within its rounding), and the iterate stays exactly invariant
    under complement and reversal."""
    p = ba.PREC_FP64 if prec == "fp64" else ba.PREC_FP32_LOG
    ns, ds = [9, 12, 11, 12], [0.64, 0.8, 0.9, 0.96]
    (lp_f, lo_f, hi_f), (lp_o, lo_o, hi_o) = stream_pair(ba, ns, ds, p, 12)
    tl, tb = (1e-12, 1e-12) if prec == "fp64" else (1e-4, 1e-5)
    assert np.max(np.abs(lp_f - lp_o)) < tl
    assert np.max(np.abs(lo_f - lo_o)) < tb and np.max(np.abs(hi_f - hi_o)) < tb
    off = 0
    for n in ns:
        x = np.arange(1 << n)
        rv = np.zeros_like(x)
        for i in range(n):
            rv |= ((x >> i) & 1) << (n - 1 - i)
        seg = lp_o[off:off + (1 << n)]
        top = seg > seg.max() - 30.0
        assert np.max(np.abs(seg[rv] - seg)[top]) < (1e-12 if prec == "fp64" else 1e-4)
        off += 1 << n


def test_orbit_mode_rejects_non_invariant_laws(ba):
    """ba_set_symmetry(2) refuses a law that is complement-symmetric but not
    reversal-invariant (mode 1 accepts it), and any non-invariant ba_set_logp."""
    n = 6
    x = np.arange(1 << n)
    cp = x ^ ((1 << n) - 1)
    lp = inp.random_logp(n, seed=90, spread=1.0)
    lp = 0.5 * (lp + lp[cp])             # complement-invariant only
    c = ba.Context(n, 0.7, engine=ba.ENGINE_STREAM)
    c.set_logp(torch.from_numpy(lp))
    with pytest.raises(ba.BAError) as e:
        c.set_symmetry(2)
    assert e.value.code == ba.BA_EINVAL and "reversal" in str(e.value)
    c.set_symmetry(1)
    c.set_symmetry(0)
    c.set_logp(torch.from_numpy(np.full(1 << n, -n * LN2)))
    c.set_symmetry(2)
    with pytest.raises(ba.BAError):
        c.set_logp(torch.from_numpy(lp))
    c.close()


def test_orbit_scatter_n20_fp32(ba):
    """The workload size: three n = 20 FP32 instances, one stream-engine iteration
    with each scatter; the laws agree within FP32 rounding."""
    ds = [0.64, 0.8, 0.95]
    (lp_f, lo_f, hi_f), (lp_o, lo_o, hi_o) = stream_pair(ba, [20] * 3, ds, ba.PREC_FP32_LOG, 1)
    assert np.max(np.abs(lp_f - lp_o)) < 1e-4
    assert np.max(np.abs(lo_f - lo_o)) < 1e-5 and np.max(np.abs(hi_f - hi_o)) < 1e-5
