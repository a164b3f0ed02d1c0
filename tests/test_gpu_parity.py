"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars (written in each test): embedding counts bit-exact; FP64 evaluations and
bounds within 1e-9 bits (in practice ~1e-12); FP32-iterated runs certified in
FP64 within 1e-6 bits of the oracle's FP64 capacity bracket.
"""
import math

import numpy as np
import pytest
import torch

import bdc_inputs as inp
from oracle import bdc

pytestmark = pytest.mark.gpu
LN2 = math.log(2.0)
ENGINES = ("factored", "stream", "pull")


@pytest.fixture(scope="module")
def ba():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_05867_amd as m
    m.lib()  # fails loudly if the library is missing
    return m


def engine_id(ba, name):
    return {"factored": ba.ENGINE_FACTORED, "stream": ba.ENGINE_STREAM, "pull": ba.ENGINE_PULL}[name]


def chain(ctx):
    """Use the launch chain even for groups small enough for the persistent kernel
    (tests of the chain's launch plans)."""
    ctx.set_tuning(ctx_mod().TUNE_PERSISTENT, 0)
    return ctx


def ctx_mod():
    import paper_2604_05867_amd as m
    return m


def say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------------------
# counts
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11, 12, 16, 20])
def test_row_counts_bit_exact(ba, oracle_native, n):
    say("row counts n=%d" % n)
    ctx = ba.Context(n, 0.5)
    xs = inp.sample_rows(n, 64 if n >= 16 else 32, seed=n)
    want = oracle_native.rows(n, xs)
    for x, (rk_o, em_o) in zip(xs, want):
        rk, em = ctx.row_counts(int(x))
        assert np.array_equal(rk, rk_o), (n, int(x))
        assert np.array_equal(em, em_o), (n, int(x))
    ctx.close()


def test_row_counts_cap_error(ba):
    ctx = ba.Context(10, 0.5)
    with pytest.raises(ba.BAError) as e:
        ctx.row_counts(0b1010101010, cap=5)
    assert e.value.code == ba.BA_EINVAL
    with pytest.raises(ba.BAError):
        ctx.row_counts(1 << 10)
    ctx.close()


@pytest.mark.parametrize("n", [1, 4, 9, 12, 16, 20])
def test_verify_all_rows(ba, oracle_native, n):
    """Every row: sum_{|y|=k} emb = C(n,k); total nnz = 2*3^n - 2^n; min row nnz
    = n+1 (constant string); max emb = C(n, floor(n/2))."""
    say("verify n=%d" % n)
    ctx = ba.Context(n, 0.5)
    st = ctx.verify_counts()
    assert st["total_nnz"] == 2 * 3 ** n - 2 ** n
    assert st["rows_failing"] == 0
    assert st["min_row_nnz"] == n + 1
    assert st["max_emb"] == math.comb(n, n // 2)
    if n <= 12:
        csr = oracle_native.CSR(n)
        assert st["max_row_nnz"] == int(np.diff(csr.indptr).max())
    ctx.close()


# ---------------------------------------------------------------------------
# one FP64 evaluation at a shared law (sweeps, log r, D, reductions)
# ---------------------------------------------------------------------------

def oracle_eval(oracle_native, n, d, lp):
    if n <= 10:
        W = bdc.channel_dense(n, d)
        ev = bdc.evaluate(W, bdc.floor_logp(bdc.normalise_logp(lp), 700.0))
        return ev.D, ev.L, ev.U, ev.I, ev.q_scaled, float(bdc.floor_logp(bdc.normalise_logp(lp), 700.0).max())
    csr = oracle_native.CSR(n)
    D, L, U, I, q = csr.evaluate(d, lp, floor_nats=700.0, want_q=True)
    lpf = bdc.floor_logp(bdc.normalise_logp(lp), 700.0)
    return D, L, U, I, q, float(bdc.normalise_logp(lpf).max())


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("n,d,kind", [(1, 0.3, "random"), (3, 0.5, "random"), (6, 0.0, "random"),
                                      (6, 1.0, "product"), (8, 0.5, "random"), (10, 0.77, "product"),
                                      (12, 0.64, "random"), (14, 0.9, "random")])
def test_eval_matches_oracle(ba, oracle_native, engine, n, d, kind):
    say("eval n=%d d=%.2f %s %s" % (n, d, kind, engine))
    lp = inp.random_logp(n, seed=n, spread=2.0) if kind == "random" else \
        inp.product_logp(n, inp.product_bit_probs(n, seed=n))
    D_o, L_o, U_o, I_o, q_o, M_o = oracle_eval(oracle_native, n, d, lp)
    ctx = ba.Context(n, d, engine=engine_id(ba, engine))
    got = ctx.eval(torch.from_numpy(lp))
    assert abs(got["L"] - L_o / LN2) < 1e-10
    assert abs(got["U"] - U_o / LN2) < 1e-10
    assert abs(got["I"] - I_o / LN2) < 1e-10
    assert np.allclose(got["D"].cpu().numpy(), D_o, atol=1e-10, rtol=0)
    if 0.0 < d < 1.0:
        k = bdc.output_lengths(n)
        w = bdc.length_weights(n, d)[k]
        r_o = q_o * np.exp(M_o) / w
        r_g = got["r"].cpu().numpy() * math.exp(got["M"])
        assert np.allclose(r_g, r_o, rtol=1e-11, atol=0)
    ctx.close()


@pytest.mark.parametrize("engine", ENGINES)
def test_eval_uniform_closed_form_n20(ba, engine):
    """At the uniform law r(y) = C(n,k) 2^-k for every y (any n)."""
    n = 20
    say("uniform closed form n=20 %s" % engine)
    ctx = ba.Context(n, 0.8, engine=engine_id(ba, engine))
    got = ctx.eval(torch.full((1 << n,), -n * LN2, dtype=torch.float64))
    r = got["r"].cpu().numpy() * math.exp(got["M"])
    want = bdc.r_uniform(n)
    assert np.allclose(r, want, rtol=1e-12, atol=0)
    assert got["L"] <= got["U"] + 1e-12
    ctx.close()


@pytest.mark.parametrize("engine", ENGINES)
def test_eval_product_law_sampled_n20(ba, oracle_native, engine):
    """Full size n = 20 at a product input law: r at sampled outputs and D at
    sampled inputs against the oracle's closed forms (one by one)."""
    n, d = 20, 0.8
    say("product law n=20 %s" % engine)
    pi1 = inp.product_bit_probs(n, seed=17)
    lp = inp.product_logp(n, pi1)
    ctx = ba.Context(n, d, engine=engine_id(ba, engine))
    got = ctx.eval(torch.from_numpy(lp))
    M = got["M"]
    ys = inp.sample_outputs(n, 4000, seed=5)
    r_g = got["r"].cpu().numpy()[ys] * math.exp(M)
    r_o = oracle_native.product_r(n, pi1, ys)
    assert np.allclose(r_g, r_o, rtol=1e-11, atol=0)
    xs = inp.sample_rows(n, 48, seed=6)
    D_o = oracle_native.product_D(n, d, pi1, xs)
    D_g = got["D"].cpu().numpy()[xs]
    assert np.allclose(D_g, D_o, atol=1e-9, rtol=0)
    # property: the upper bound is the max of D, the lower bound below it
    assert got["U"] >= float(D_o.max()) / LN2 - 1e-9
    assert got["L"] <= got["U"]
    ctx.close()


# ---------------------------------------------------------------------------
# iterations
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("engine", list(ENGINES) + ["persistent"])
@pytest.mark.parametrize("n,d,iters", [(2, 0.5, 40), (8, 0.5, 25), (11, 0.7, 10)])
def test_fp64_iterates_match_oracle(ba, engine, n, d, iters):
    say("iterates n=%d %s" % (n, engine))
    W = bdc.channel_dense(n, d)
    ctx = ba.Context(n, d, engine=engine_id(ba, "factored" if engine == "persistent" else engine))
    if engine == "factored":
        chain(ctx)
    elif engine == "persistent":
        ctx.set_tuning(ba.TUNE_PERSISTENT, 2)
    ctx.step(iters)
    lp_g = ctx.get_logp().cpu().numpy()
    lp_o = bdc.ba_iterate(W, bdc.uniform_logp(n), iters)
    assert np.max(np.abs(lp_g - lp_o)) < 1e-10
    lo, hi = ctx.bounds()
    L_o, U_o = bdc.certify(W, lp_o)
    assert abs(lo[0] - L_o) < 1e-10 and abs(hi[0] - U_o) < 1e-10
    ctx.close()


@pytest.mark.parametrize("path", ["chain", "persistent"])
def test_config1_n8_to_1e9(ba, path):
    """n = 8, d = 0.5, FP64 until the gap is below 1e-9 bits, against the oracle's
    BA with the same stopping rule (Section 2.3), with the launch chain and with
    the persistent launch (which tests the gap of every iterate in the kernel)."""
    n, d = 8, 0.5
    W = bdc.channel_dense(n, d)
    res = bdc.ba(W, n, tol_bits=1e-9, max_iters=20000)
    ctx = ba.Context(n, d)
    if path == "chain":
        chain(ctx)
    done = ctx.run(1e-9, 20000)
    lo, hi, its = ctx.best_bounds()
    say("C1: gpu iters=%d oracle iters=%d" % (its[0], res.iters))
    assert its[0] == res.iters
    assert abs(lo[0] - res.lower_bits) < 1e-9 and abs(hi[0] - res.upper_bits) < 1e-9
    assert hi[0] - lo[0] < 1e-9
    assert done >= res.iters
    ctx.close()


def oracle_ba_csr(csr, d, tol_bits, max_iters):
    """The BA loop of Section 2.3 on the C oracle's sparse channel, with log p
    floored at 700 nats below its max (the optimum has zero-probability inputs,
    so unfloored iterates underflow FP64 after a few thousand iterations)."""
    lp = bdc.uniform_logp(csr.n)
    for t in range(max_iters + 1):
        D, L, U, I, _ = csr.evaluate(d, lp, floor_nats=700.0)
        if (U - L) / LN2 < tol_bits or t == max_iters:
            return L / LN2, U / LN2, t
        lp = bdc.floor_logp(bdc.normalise_logp(lp) + D - L, 700.0)


def test_fp32_log_domain_certified(ba, oracle_native):
    """FP32 iterates, FP64 certification: certified gap < 1e-6 bits and the
    certified bracket intersects the oracle's FP64 bracket."""
    n, d = 10, 0.8
    L_o, U_o, t_o = oracle_ba_csr(oracle_native.CSR(n), d, 1e-8, 100000)
    ctx = ba.Context(n, d, prec=ba.PREC_FP32_LOG, cert_every=50)
    done = ctx.run(1e-6, 60000)
    lo, hi, its = ctx.best_bounds()
    say("fp32: iters=%d L=%.12f U=%.12f ref=[%.12f, %.12f] (%d)" % (done, lo[0], hi[0], L_o, U_o, t_o))
    assert hi[0] - lo[0] < 1e-6
    assert lo[0] <= U_o + 1e-12 and L_o <= hi[0] + 1e-12
    assert abs(lo[0] - L_o) < 1e-6
    ctx.close()


@pytest.mark.parametrize("engine", ENGINES)
def test_batch_equals_singles(ba, engine):
    ns = [6, 8, 6, 7, 8]
    ds = [0.3, 0.5, 0.9, 0.64, 0.96]
    ctx = ba.Context(ns, ds, prec=ba.PREC_FP64, engine=engine_id(ba, engine))
    ctx.step(15)
    lo, hi = ctx.bounds()
    lp_all = ctx.get_logp().cpu().numpy()
    off = 0
    for i, (n, d) in enumerate(zip(ns, ds)):
        s = ba.Context(n, d, engine=engine_id(ba, engine))
        s.step(15)
        l1, h1 = s.bounds()
        assert abs(l1[0] - lo[i]) < 1e-12 and abs(h1[0] - hi[i]) < 1e-12
        assert np.allclose(s.get_logp().cpu().numpy(), lp_all[off:off + (1 << n)], atol=1e-12)
        off += 1 << n
        s.close()
    ctx.close()


def test_engines_agree_fp32_batch(ba):
    ns = [10, 12]
    ds = [0.64, 0.96]
    out = []
    for eng in (ba.ENGINE_FACTORED, ba.ENGINE_STREAM):
        c = ba.Context(ns, ds, prec=ba.PREC_FP32_LOG, engine=eng)
        c.step(20)
        out.append(c.get_logp().cpu().numpy())
        c.close()
    assert np.max(np.abs(out[0] - out[1])) < 1e-3


def test_symmetry_of_iterates_n16(ba):
    """Theorem 4: from uniform, p(cpl x) = p(x) = p(rev x) at every iteration."""
    n = 16
    ctx = ba.Context(n, 0.7)
    ctx.step(30)
    lp = ctx.get_logp().cpu().numpy()
    x = np.arange(1 << n)
    cp = x ^ ((1 << n) - 1)
    rv = np.zeros_like(x)
    for i in range(n):
        rv |= ((x >> i) & 1) << (n - 1 - i)
    assert np.max(np.abs(lp[cp] - lp)) < 1e-9
    assert np.max(np.abs(lp[rv] - lp)) < 1e-9
    ctx.close()


def test_set_get_logp_and_numeric_errors(ba):
    n = 6
    ctx = ba.Context(n, 0.5)
    lp = torch.from_numpy(inp.random_logp(n, seed=3))
    ctx.set_logp(lp)
    back = ctx.get_logp().cpu().numpy()
    assert np.allclose(back, bdc.normalise_logp(lp.numpy()), atol=1e-13)
    bad = lp.clone()
    bad[5] = float("nan")
    with pytest.raises(ba.BAError) as e:
        ctx.set_logp(bad)
    assert e.value.code == ba.BA_ENUMERIC
    ctx.close()


# ---------------------------------------------------------------------------
# gradients and mirror ascent
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("engine", ENGINES)
def test_gradients_match_oracle(ba, engine):
    n, d = 8, 0.8
    theta = inp.theta_normal(n, seed=0, sigma=0.1)
    I_o, g_o, gd_o = bdc.info_and_grads(n, d, theta)
    ctx = ba.Context(n, d, engine=engine_id(ba, engine))
    I, g, gd = ctx.grad(torch.from_numpy(theta))
    assert abs(I - I_o) < 1e-11
    assert np.allclose(g.cpu().numpy(), g_o, atol=1e-12)
    assert abs(gd - gd_o) < 1e-10
    ctx.close()


def test_autograd_function(ba):
    n, d = 6, 0.6
    ctx = ba.Context(n, d)
    theta = torch.from_numpy(inp.theta_normal(n, seed=1, sigma=0.2)).requires_grad_(True)
    dd = torch.tensor(d, dtype=torch.float64, requires_grad=True)
    I = ba.BAInfo.apply(theta, dd, ctx)
    I.backward()
    I_o, g_o, gd_o = bdc.info_and_grads(n, d, theta.detach().numpy())
    assert abs(I.item() - I_o) < 1e-11
    assert np.allclose(theta.grad.numpy(), g_o, atol=1e-12)
    assert abs(dd.grad.item() - gd_o) < 1e-10
    ctx.close()


def test_mirror_ascent_unit_step_is_ba(ba):
    n, d = 7, 0.65
    theta = inp.theta_normal(n, seed=2, sigma=0.3)
    ctx = ba.Context(n, d)
    th = ctx.mirror_ascent(torch.from_numpy(theta), 1.0, 12).cpu().numpy()
    th_o = bdc.mirror_ascent(n, d, theta, 1.0, 12)
    assert np.allclose(bdc.normalise_logp(th), bdc.normalise_logp(th_o), atol=1e-11)
    th2 = ctx.mirror_ascent(torch.from_numpy(theta), 2.0, 5).cpu().numpy()
    th2_o = bdc.mirror_ascent(n, d, theta, 2.0, 5)
    assert np.allclose(bdc.normalise_logp(th2), bdc.normalise_logp(th2_o), atol=1e-11)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replay_matches_eager(ba, prec):
    """ba_run replaying a captured graph (many replays with host reads between
    them) gives the same iterates as eager launches; the factored engine has no
    atomics, so the results are bitwise equal."""
    ns = [8, 10, 8]
    ds = [0.5, 0.7, 0.9]
    p = ba.PREC_FP64 if prec == "fp64" else ba.PREC_FP32_LOG
    out = []
    s = torch.cuda.Stream()
    c = ba.Context(ns, ds, prec=p, cert_every=20, stream=s)
    start = torch.cat([torch.full((1 << n,), 0.0, dtype=torch.float64) for n in ns])
    for graphs in (False, True):
        # the same starting state for both runs
        c.set_graphs(graphs)
        with torch.cuda.stream(s):
            c.set_logp(start)
            done = c.run(1e-7, 400)
            lo, hi, its = c.best_bounds()
            lp = c.get_logp().cpu().numpy()
        s.synchronize()
        out.append((done, lo, hi, its, lp))
    c.close()
    assert out[0][0] == out[1][0] and out[0][3] == out[1][3]
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]
    assert np.array_equal(out[0][4], out[1][4])


def test_graph_needs_a_stream(ba):
    c = ba.Context(6, 0.5)
    c.set_graphs(True)
    if c.stream.cuda_stream == 0:
        with pytest.raises(ba.BAError) as e:
            c.run(1e-6, 10)
        assert e.value.code == ba.BA_ESTATE
    c.close()


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 12, 13, 16, 17, 20])
def test_factored_fusion_settings_agree(ba, n):
    """One, two, four and eight input positions per launch, the last four and the
    first eight forward positions in one launch, and (n = 20) the backward sweep as
    twelve positions then eight, give the same evaluation (all against the oracle
    for n <= 8)."""
    d = 0.6
    lp = inp.random_logp(n, seed=40 + n, spread=2.0)
    say("fusion settings n=%d" % n)
    out = []
    for fuse in (0, 1, 2, 3, 4, 5, 6, 7):
        c = ba.Context(n, d)
        c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        got = c.eval(torch.from_numpy(lp))
        out.append((got["L"], got["U"], got["r"].cpu().numpy(), got["D"].cpu().numpy()))
        c.close()
    for o in out[1:]:
        assert abs(out[0][0] - o[0]) < 1e-12 and abs(out[0][1] - o[1]) < 1e-12
        assert np.allclose(out[0][2], o[2], rtol=1e-13, atol=0)
        assert np.allclose(out[0][3], o[3], atol=1e-12)
    # eight positions per launch are two four-position steps with the same sums in
    # the same order: bitwise equal
    c = ba.Context(n, d)
    same = []
    for fuse in (2, 3, 4, 5, 6):
        c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        got = c.eval(torch.from_numpy(lp))
        same.append((got["L"], got["U"], got["r"].cpu().numpy(), got["D"].cpu().numpy()))
    c.close()
    assert np.array_equal(same[0][3], same[1][3]) and same[0][0] == same[1][0] and same[0][1] == same[1][1]
    # the first eight forward positions in one launch are two four-position steps
    assert np.array_equal(same[2][2], same[3][2]) and np.array_equal(same[2][3], same[3][3])
    # twelve backward positions in one launch are three four-position steps
    assert np.array_equal(same[3][3], same[4][3]) and same[3][0] == same[4][0] and same[3][1] == same[4][1]
    if n <= 8:
        ev = bdc.evaluate(bdc.channel_dense(n, d), lp)
        assert abs(out[1][0] - ev.L / LN2) < 1e-11


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8, 11, 16])
def test_four_position_backward_iterates(ba, n):
    """Iterations with four positions per backward launch (D fused into the last
    one) equal those with two, FP64."""
    out = []
    for fuse in (1, 2):
        c = chain(ba.Context(n, 0.65))
        c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        c.step(20)
        out.append((c.get_logp().cpu().numpy(), c.bounds()))
        c.close()
    assert np.max(np.abs(out[0][0] - out[1][0])) < 1e-12
    assert abs(out[0][1][0][0] - out[1][1][0][0]) < 1e-12 and abs(out[0][1][1][0] - out[1][1][1][0]) < 1e-12


@pytest.mark.parametrize("n,prec", [(12, "fp64"), (13, "fp64"), (17, "fp64"), (20, "fp32"), (19, "fp32")])
def test_eight_position_backward_is_bitwise_four(ba, n, prec):
    """Eight positions per backward launch (two four-position steps through LDS)
    give bitwise the iterates and bounds of four positions per launch."""
    p = ba.PREC_FP64 if prec == "fp64" else ba.PREC_FP32_LOG
    ns = [n] * 3 if prec == "fp32" else [n]
    ds = [0.64, 0.8, 0.95] if prec == "fp32" else [0.7]
    # one context (the same H), reset to the uniform law between the two runs
    c = chain(ba.Context(ns, ds, prec=p))
    X = sum(1 << m for m in ns)
    start = torch.tensor(np.concatenate([np.full(1 << m, -m * LN2) for m in ns]))
    out = []
    for fuse in (2, 3):
        c.set_logp(start)
        c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        c.step(4)
        out.append((c.get_logp().cpu().numpy(), c.bounds()))
    c.close()
    assert out[0][0].shape == (X,)
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_twelve_position_backward_iterates(ba, prec):
    """At n = 20 the backward sweep as twelve positions then eight with D (launch
    plan level 6) gives the iterates and bounds of level 5 (eight, eight, four with
    D): the same G; only the grouping of the D records' sums differs."""
    n = 20
    p = ba.PREC_FP64 if prec == "fp64" else ba.PREC_FP32_LOG
    ns = [n] * 3 if prec == "fp32" else [n]
    ds = [0.64, 0.8, 0.95] if prec == "fp32" else [0.7]
    say("twelve-position backward %s" % prec)
    c = chain(ba.Context(ns, ds, prec=p))
    start = torch.tensor(np.concatenate([np.full(1 << m, -m * LN2) for m in ns]))
    out = []
    for fuse in (5, 6):
        c.set_logp(start)
        c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        c.step(4)
        out.append((c.get_logp().cpu().numpy(), c.bounds()))
    c.close()
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert np.max(np.abs(out[0][0] - out[1][0])) < tol
    for k in range(len(ns)):
        assert abs(out[0][1][0][k] - out[1][1][0][k]) < tol and abs(out[0][1][1][k] - out[1][1][1][k]) < tol


@pytest.mark.parametrize("seed", [0, 1])
def test_twelve_position_forward_is_bitwise(ba, seed):
    """At n = 20 (FP32) the forward positions 8-19 in one launch per leaf of F_8
    (launch plan level 7: the leaf's ancestor rows recomputed in its block) give
    bitwise the iterates and bounds of level 6 (positions 8-11, 12-15 and 16-19 in
    three launches): every value is the same sum in the same order."""
    n = 20
    ns, ds = [n] * 3, [0.64, 0.8, 0.95]
    say("twelve-position forward seed=%d" % seed)
    c = chain(ba.Context(ns, ds, prec=ba.PREC_FP32_LOG))
    start = torch.tensor(np.concatenate([inp.random_logp(n, seed=70 + 3 * seed + k, spread=3.0)
                                         for k in range(3)]))
    out = []
    for fuse in (6, 7):
        c.set_logp(start)
        c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        c.step(3)
        out.append((c.get_logp().cpu().numpy(), c.bounds()))
    c.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


@pytest.mark.parametrize("n,prec", [(12, "fp64"), (17, "fp64"), (20, "fp32"), (20, "fp64")])
def test_first_eight_forward_is_bitwise_four(ba, n, prec):
    """The first eight forward positions in one launch (two four-position steps
    through LDS, with the pending update fused in) give bitwise the iterates and
    bounds of two four-position launches."""
    p = ba.PREC_FP64 if prec == "fp64" else ba.PREC_FP32_LOG
    ns = [n] * 3 if prec == "fp32" else [n]
    ds = [0.64, 0.8, 0.95] if prec == "fp32" else [0.7]
    say("first eight forward n=%d %s" % (n, prec))
    c = chain(ba.Context(ns, ds, prec=p))
    start = torch.tensor(np.concatenate([np.full(1 << m, -m * LN2) for m in ns]))
    out = []
    for fuse in (4, 5):
        c.set_logp(start)
        c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        c.step(4)
        out.append((c.get_logp().cpu().numpy(), c.bounds()))
    c.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


@pytest.mark.parametrize("n,prec,sym", [(16, "fp32", False), (13, "fp64", False), (16, "fp32", True),
                                        (20, "fp32", False), (20, "fp32", True)])
def test_freeze_flag_skip_is_bitwise(ba, n, prec, sym):
    """Until a gap tolerance is set (ba_run) no instance can be frozen by one, and the
    sweep kernels skip reading the frozen flag: the iterates of step() then equal,
    bit for bit, those of the same iterations run by ba_run (flag read) in the same
    context.  After ba_run has frozen the instances, step() leaves them untouched."""
    p = ba.PREC_FP64 if prec == "fp64" else ba.PREC_FP32_LOG
    ns, ds = [n, n], [0.6, 0.9]
    say("freeze flag skip n=%d %s sym=%d" % (n, prec, sym))
    c = chain(ba.Context(ns, ds, prec=p))
    start = torch.tensor(np.concatenate([np.full(1 << m, -m * LN2) for m in ns]))
    c.set_logp(start)
    if sym:
        c.set_symmetry(True)
    c.step(6)
    skipped = c.get_logp().cpu().numpy()
    c.set_logp(start)
    assert c.run(1e-12, 6) == 6
    read = c.get_logp().cpu().numpy()
    assert np.array_equal(skipped, read)
    # a gap every iterate meets: frozen after the first chunk, then step() is a no-op
    c.run(20.0, 10)
    frozen = c.get_logp().cpu().numpy()
    c.step(3)
    assert np.array_equal(frozen, c.get_logp().cpu().numpy())
    c.close()


def test_four_position_backward_n20_fp32(ba):
    ds = [0.64, 0.8, 0.95]
    out = []
    for fuse in (1, 2):
        c = ba.Context([20] * 3, ds, prec=ba.PREC_FP32_LOG)
        c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        c.step(5)
        out.append((c.get_logp().cpu().numpy(), c.bounds()))
        c.close()
    # FP32 iterates of two summation orders: the laws differ by FP32 rounding
    # (~1e-6 nats in log p), which moves the FP64-certified bounds by ~1e-6 bits
    assert np.max(np.abs(out[0][0] - out[1][0])) < 1e-4
    assert np.max(np.abs(np.array(out[0][1][0]) - np.array(out[1][1][0]))) < 5e-6
    assert np.max(np.abs(np.array(out[0][1][1]) - np.array(out[1][1][1]))) < 5e-6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_update_is_bitwise_separate(ba, prec):
    """Within one step call the update of each iteration but the last runs inside
    the next iteration's first forward launch; the iterates and bounds equal those
    of one-iteration calls (separate update launches) bit for bit, with and without
    a step eta.  (FP32 iterates at launch plan levels 6-8 shift by the max in
    between instead: test_fp32_update_by_max_matches_normalised, so FP32 runs at
    level 5 here.)"""
    p = ba.PREC_FP64 if prec == "fp64" else ba.PREC_FP32_LOG
    ns, ds = ([12, 14], [0.6, 0.9]) if prec == "fp64" else ([16, 17], [0.7, 0.95])
    # one context, reset between runs
    c = chain(ba.Context(ns, ds, prec=p))
    if prec == "fp32":
        c.set_tuning(ba.TUNE_FACTORED_FUSE, 5)
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
    c.close()


@pytest.mark.parametrize("n,d", [(20, 0.64), (20, 0.8), (16, 0.8)])
def test_fp32_update_by_max_matches_normalised(ba, n, d):
    """FP32 BA iterations (n = 20 and 16) within one step call shift log p by the max
    of log p + D (from the D launch's block maxima, no final-record launch) instead of
    normalising; the call's last update normalises.  The result equals that of
    one-iteration calls (every update normalised) to FP32 rounding: log p (magnitude
    ~14, ulp ~1e-6) within 4e-5 after 7 iterations, the FP64-certified bounds within
    1e-6 bits; and one final-record launch ran for the 7 iterations."""
    say("fp32 update by max n=%d d=%g" % (n, d))
    c = chain(ba.Context([n], [d], prec=ba.PREC_FP32_LOG))
    start = torch.tensor(np.full(1 << n, -n * LN2))
    out = []
    for per_call in (1, 7):
        c.set_logp(start)
        for _ in range(7 // per_call):
            c.step(per_call)
        out.append((c.get_logp().cpu().numpy(), c.bounds()))
    c.set_logp(start)
    t = c.time_kernels(7)
    c.close()
    assert t["reduce"][1] == 1
    assert np.max(np.abs(out[0][0] - out[1][0])) < 4e-5
    assert abs(out[0][1][0][0] - out[1][1][0][0]) < 1e-6 and abs(out[0][1][1][0] - out[1][1][1][0]) < 1e-6


@pytest.mark.parametrize("per_call", [1, 2, 3, 7])
def test_fused_next_iteration_matches_plan7(ba, per_call):
    """Launch plan level 8 (n = 20, FP32): inside a step call, from the second
    iteration on, each D launch but the last also makes the next iteration's update
    (a shift by the previous iteration's max of log p + D) and first eight forward
    positions.  The iterates equal those of level 7 (shift by the current max) to FP32
    rounding: log p within 4e-5 and the FP64-certified bounds within 1e-6 bits after 7
    iterations in calls of 1, 2, 3 or 7; with 7 per call, 9 forward launches (first8 and
    k_fwd_stage12 in iterations 0 and 1, then k_fwd_stage12 alone) and one record
    reduction ran."""
    n = 20
    ns, ds = [n] * 3, [0.64, 0.8, 0.95]
    say("fused next iteration per_call=%d" % per_call)
    c = chain(ba.Context(ns, ds, prec=ba.PREC_FP32_LOG))
    start = torch.tensor(np.concatenate([inp.random_logp(n, seed=90 + k, spread=3.0) for k in range(3)]))
    out = []
    for fuse in (7, 8):
        c.set_logp(start)
        c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        done = 0
        while done < 7:
            k = min(per_call, 7 - done)
            c.step(k)
            done += k
        out.append((c.get_logp().cpu().numpy(), c.bounds()))
    if per_call == 7:
        c.set_logp(start)
        t = c.time_kernels(7)
        assert t["sweep1"][1] == 9 and t["sweep2"][1] == 14 and t["reduce"][1] == 1
    c.close()
    assert np.all(np.isfinite(out[1][0]))
    assert np.max(np.abs(out[0][0] - out[1][0])) < 4e-5
    for k in range(3):
        assert abs(out[0][1][0][k] - out[1][1][0][k]) < 1e-6 and abs(out[0][1][1][k] - out[1][1][1][k]) < 1e-6


# launch plans 6-8 at lengths other than 20 (FP32): forward launches at level 5 per
# iteration (first8 and the rest), backward launches at level 8 per iteration
PLAN8_LAUNCHES = {12: (2, 2), 13: (3, 3), 14: (3, 3), 15: (4, 4), 16: (3, 2), 17: (4, 3), 18: (4, 3), 19: (5, 4)}


@pytest.mark.parametrize("n", sorted(PLAN8_LAUNCHES))
def test_fused_next_iteration_other_n(ba, n):
    """Launch plan levels 6-8 at lengths other than 20 (FP32, three instances): the
    backward launches stop at position 8 for one eight-position D launch, which writes
    the block maxima of log p + D (the next update shifts by the max; no final-record
    launch) and at level 8 also makes the next iteration's update and first eight
    forward positions.  The iterates equal those of level 5 (every update normalised)
    to FP32 rounding after 7 iterations in calls of 1, 3 or 7 (log p within 4e-5, the
    FP64-certified bounds within 1e-6 bits); with 7 per call, level 8 runs the first
    eight forward positions as their own launch in iterations 0 and 1 only, its
    backward launches per iteration, and one record reduction."""
    ns, ds = [n] * 3, [0.64, 0.8, 0.95]
    say("plan 8 at n=%d" % n)
    c = chain(ba.Context(ns, ds, prec=ba.PREC_FP32_LOG))
    start = torch.tensor(np.concatenate([inp.random_logp(n, seed=120 + k, spread=3.0) for k in range(3)]))
    ref = None
    for fuse in (5, 6, 8):
        c.set_tuning(ba.TUNE_FACTORED_FUSE, fuse)
        for per_call in ((1,) if fuse == 5 else (1, 3, 7)):
            c.set_logp(start)
            done = 0
            while done < 7:
                k = min(per_call, 7 - done)
                c.step(k)
                done += k
            got = (c.get_logp().cpu().numpy(), c.bounds())
            if ref is None:
                ref = got
                continue
            assert np.all(np.isfinite(got[0]))
            assert np.max(np.abs(got[0] - ref[0])) < 4e-5, (fuse, per_call)
            for j in range(3):
                assert abs(got[1][0][j] - ref[1][0][j]) < 1e-6 and abs(got[1][1][j] - ref[1][1][j]) < 1e-6
    c.set_logp(start)
    t = c.time_kernels(7)
    c.close()
    f5, b8 = PLAN8_LAUNCHES[n]
    assert t["sweep1"][1] == 7 * f5 - 5 and t["sweep2"][1] == 7 * b8 and t["reduce"][1] == 1


@pytest.mark.parametrize("n", [16, 20])
def test_fp32_default_plan_tracks_fp64_iterates(ba, n):
    """The default plan's FP32-only launches (first eight positions, the
    twelve-position launches at n = 20, the D launch fused with the next update)
    against the FP64 launch chain, which the oracle pins: three instances from a
    random full-support law, 30 iterations in calls of 10, both at the 80-nat floor.
    log p agrees to FP32 accuracy on the inputs within 30 nats of the maximum (the
    mass the bounds depend on): within 2e-4 nats (measured 2-3e-5 after 30
    iterations of ~1e-7 relative rounding on values up to ~40); the FP64-certified
    bounds of the two iterates: L within 1e-6 bits, U = max D, which moves with the
    iterate's rounding at its maximising input, within 2e-6 bits (measured up to
    7e-7)."""
    ns, ds = [n] * 3, [0.64, 0.8, 0.95]
    say("fp32 default plan against fp64 n=%d" % n)
    start = torch.tensor(np.concatenate([inp.random_logp(n, seed=150 + k, spread=3.0) for k in range(3)]))
    out = []
    for p in (ba.PREC_FP32_LOG, ba.PREC_FP64):
        c = chain(ba.Context(ns, ds, prec=p))
        c.set_floor(80.0)
        c.set_logp(start)
        for _ in range(3):
            c.step(10)
        out.append((c.get_logp().cpu().numpy().reshape(3, 1 << n), c.bounds()))
        c.close()
    for k in range(3):
        lp32, lp64 = out[0][0][k], out[1][0][k]
        top = lp64 > lp64.max() - 30.0
        err = float(np.max(np.abs(lp32 - lp64)[top]))
        say("n=%d d=%.2f: max |log p32 - log p64| = %.2e, bounds %.2e %.2e" % (
            n, ds[k], err, out[0][1][0][k] - out[1][1][0][k], out[0][1][1][k] - out[1][1][1][k]))
        assert err < 2e-4
        assert abs(out[0][1][0][k] - out[1][1][0][k]) < 1e-6 and abs(out[0][1][1][k] - out[1][1][1][k]) < 2e-6


def test_symmetric_other_n_keeps_symmetric_kernels(ba):
    """With ba_set_symmetry at n = 16 (FP32, launch plan 8) the complement-symmetric
    kernels run (the half plan is the twelve-position plan of n = 20 only): the
    iterate stays exactly complement-invariant and agrees with the full plan to FP32
    rounding."""
    n, ds = 16, [0.64, 0.9]
    out = []
    for sym in (False, True):
        c = chain(ba.Context([n] * 2, ds, prec=ba.PREC_FP32_LOG))
        if sym:
            c.set_symmetry(True)
        c.step(7)
        out.append(c.get_logp().cpu().numpy().reshape(2, 1 << n))
        c.close()
    for k in range(2):
        assert np.array_equal(out[1][k], out[1][k][::-1])
    assert np.max(np.abs(out[0] - out[1])) < 4e-5


@pytest.mark.parametrize("path", ["chain", "persistent"])
def test_fused_update_stops_at_tolerance(ba, path):
    """FP64 iterates stop at the first iterate whose gap is below the tolerance,
    also when that test is made inside a fused first forward launch, or inside the
    persistent launch's loop (ba_run, eager and graph-replayed)."""
    n, d, tol = 10, 0.5, 1e-2
    setp = chain if path == "chain" else (lambda c: c)
    # reference: one iteration per call (separate update launches, no stop test)
    ref = setp(ba.Context(n, d))
    k = 0
    while k < 3000:
        ref.step(1)
        k += 1
        lo, hi = ref.bounds()  # certified bounds of iterate k
        if hi[0] - lo[0] < tol:
            break
    assert hi[0] - lo[0] < tol and k > 40  # several chunks of the FP64 run loop
    lp_ref = ref.get_logp().cpu().numpy()
    ref.close()
    for graphs in (False, True):
        s = torch.cuda.Stream()
        c = setp(ba.Context(n, d, stream=s))
        c.set_graphs(graphs)
        with torch.cuda.stream(s):
            c.run(tol, 3000)
            lo, hi = c.bounds()
            its = c.best_bounds()[2]
            lp = c.get_logp().cpu().numpy()
        s.synchronize()
        c.close()
        # stopped at iterate k (its bounds tested, no update made)
        assert its[0] == k
        assert hi[0] - lo[0] < tol
        assert np.max(np.abs(lp - lp_ref)) < 1e-10


@pytest.mark.parametrize("case", ["fp64_batch", "fp32_n20", "exact"])
def test_init_is_deterministic_across_contexts(ba, case):
    """H(x) and Hd(x) (the init pass over every nonzero, Section 3's per-input
    constant) are summed with order-independent fixed-point integer atomics, so two
    contexts of the same instances give bitwise-identical H, iterates, certified
    bounds and gradients (the factored engine has no atomics in its sweeps)."""
    if case == "fp64_batch":
        kw = dict(n=[12, 9, 12], d=[0.64, 0.3, 0.9], prec=ba.PREC_FP64)
    elif case == "fp32_n20":
        kw = dict(n=[20, 20], d=[0.64, 0.95], prec=ba.PREC_FP32_LOG)
    else:
        kw = dict(n=[10, 10], d=None, prec=ba.PREC_FP64, k=[3, 7])
    res = []
    for _ in range(2):
        c = ba.Context(kw["n"], kw["d"], prec=kw["prec"], k=kw.get("k"))
        c.step(25)
        lo, hi = c.bounds()
        lp = c.get_logp().cpu().numpy()
        grad = None
        if case == "fp64_batch":
            theta = torch.from_numpy(inp.theta_normal(12, seed=5, sigma=0.3))
            I, g, dd = c.grad(theta)
            grad = (I, dd, g.cpu().numpy())
        res.append((lo, hi, lp, grad))
        c.close()
    assert res[0][0] == res[1][0] and res[0][1] == res[1][1]
    assert np.array_equal(res[0][2], res[1][2])
    if res[0][3] is not None:
        assert res[0][3][0] == res[1][3][0] and res[0][3][1] == res[1][3][1]
        assert np.array_equal(res[0][3][2], res[1][3][2])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_concurrent_group_branches_are_bitwise(ba, prec):
    """ba_run's captured chunk with one graph branch per group (n) gives bitwise the
    iterates, certified and best bounds of the same chunk captured group after group,
    and of eager launches: the groups share no arrays."""
    ns = [10, 12, 14, 10, 12, 14]
    ds = [0.64, 0.7, 0.8, 0.9, 0.95, 0.66]
    p = ba.PREC_FP64 if prec == "fp64" else ba.PREC_FP32_LOG
    out = []
    for mode in ("eager", "sequential", "concurrent"):
        s = torch.cuda.Stream()
        c = ba.Context(ns, ds, prec=p, cert_every=25, stream=s)
        c.set_graphs(mode != "eager")
        c.set_tuning(ba.TUNE_CONCURRENT_GROUPS, 1 if mode == "concurrent" else 0)
        with torch.cuda.stream(s):
            done = c.run(1e-5, 300)
            lo, hi, its = c.best_bounds()
            clo, chi = c.bounds()
            lp = c.get_logp().cpu().numpy()
        s.synchronize()
        out.append((done, lo, hi, its, clo, chi, lp))
        c.close()
    for o in out[1:]:
        assert o[0] == out[0][0] and o[3] == out[0][3]
        assert o[1] == out[0][1] and o[2] == out[0][2] and o[4] == out[0][4] and o[5] == out[0][5]
        assert np.array_equal(o[6], out[0][6])


PERSIST_CASES = {
    "fp64": dict(n=[3, 7, 12, 9], d=[0.1, 0.64, 0.8, 0.99], prec="fp64"),
    "fp64_eta": dict(n=[10, 12], d=[0.7, 0.9], prec="fp64", eta=1.7),
    "fp32": dict(n=[10, 13, 12, 13], d=[0.64, 0.8, 0.96, 0.5], prec="fp32"),
    "exact": dict(n=[11, 11, 6], k=[4, 9, 6], prec="fp64"),
    "floor": dict(n=[8], d=[0.8], prec="fp64", floor=50.0, iters=1500),
    "mixed": dict(n=[12, 14, 13, 16], d=[0.7, 0.7, 0.9, 0.9], prec="fp64"),
}


@pytest.mark.parametrize("case", sorted(PERSIST_CASES))
def test_persistent_equals_chain(ba, case):
    """The persistent launch (one block per instance iterating in LDS, one position
    per stage) against the launch chain (four or eight positions per launch): the
    same iteration up to the order of additions.  FP64: iterates within 1e-11 nats
    and certified bounds within 1e-11 bits; FP32: within FP32 rounding (iterates
    1e-4 nats, certified bounds 1e-5 bits).  Groups too large for LDS (n = 14, 16
    in "mixed") take the chain on both sides."""
    kw = PERSIST_CASES[case]
    p = ba.PREC_FP64 if kw["prec"] == "fp64" else ba.PREC_FP32_LOG
    iters = kw.get("iters", 40)
    say("persistent vs chain: %s" % case)
    out = []
    for persistent in (0, 2):
        c = ba.Context(kw["n"], kw.get("d", None), prec=p, k=kw.get("k"))
        c.set_tuning(ba.TUNE_PERSISTENT, persistent)
        if "eta" in kw:
            c.set_step(kw["eta"])
        if "floor" in kw:
            c.set_floor(kw["floor"])
        c.step(iters // 2)
        c.step(iters - iters // 2)
        lo, hi = c.bounds()
        out.append((c.get_logp().cpu().numpy(), lo, hi, c.best_bounds()[2]))
        c.close()
    tl, tb = (1e-11, 1e-11) if kw["prec"] == "fp64" else (1e-4, 1e-5)
    assert np.max(np.abs(out[0][0] - out[1][0])) < tl
    assert np.max(np.abs(np.array(out[0][1]) - np.array(out[1][1]))) < tb
    assert np.max(np.abs(np.array(out[0][2]) - np.array(out[1][2]))) < tb
    assert out[0][3] == out[1][3] == [iters] * len(kw["n"])
