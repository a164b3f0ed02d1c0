"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests touches the GPU.  Each test names the fact it checks; a
mistake anywhere in the oracle (a dropped term, a wrong sign, an index off by
one, a transposed operand) should fail at least one of them.
"""
import math
import os

import numpy as np
import pytest

import bdc_inputs as inp
from oracle import bdc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LN2 = math.log(2.0)


def paper_values():
    vals = {}
    for line in open(os.path.join(GOLDEN, "paper_values.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, val, _cite = line.split()
        vals[key] = float(val)
    return vals


def bits_of(x, n):
    return [(x >> (n - 1 - i)) & 1 for i in range(n)]


def cpl(x, n):
    return x ^ ((1 << n) - 1)


def rev(x, n):
    out = 0
    for i in range(n):
        out = (out << 1) | ((x >> i) & 1)
    return out


# --------------------------------------------------------------------------
# Embedding counts
# --------------------------------------------------------------------------

def test_emb_n2_matches_hand_fixture(oracle_native):
    rows = {}
    for line in open(os.path.join(GOLDEN, "emb_n2.txt")):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        rows[int(parts[0], 2)] = [int(v) for v in parts[1:]]
    E = bdc.emb_dense(2)
    for x, want in rows.items():
        assert E[x].tolist() == want
        rk, em = oracle_native.row(2, x)
        dense = [0] * 7
        for r, e in zip(rk, em):
            dense[int(r)] = int(e)
        assert dense == want


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_emb_subsets_equals_position_recursion(n):
    """Two independent definitions: subset enumeration (emb_dense) and the
    position recursion 'x_0 deleted or matched' (emb_brute)."""
    E = bdc.emb_dense(n)
    for x in range(1 << n):
        xb = bits_of(x, n)
        for r in range(E.shape[1]):
            yb, k = bdc.unrank(r)
            assert E[x, r] == bdc.emb_brute(bits_of(yb, k), xb)


@pytest.mark.parametrize("n", [1, 3, 5, 8, 10])
def test_length_sums_are_binomial(n):
    """sum_{|y|=k} emb(y,x) = C(n,k): each of the C(n,k) position sets of size k
    yields exactly one y of length k."""
    E = bdc.emb_dense(n)
    k = bdc.output_lengths(n)
    for kk in range(n + 1):
        assert np.all(E[:, k == kk].sum(axis=1) == math.comb(n, kk))


@pytest.mark.parametrize("n", [16, 20])
def test_length_sums_sampled_rows_native(oracle_native, n):
    xs = inp.sample_rows(n, 24, seed=11)
    for (rk, em) in oracle_native.rows(n, xs):
        k = np.floor(np.log2(rk.astype(np.int64) + 1)).astype(int)
        for kk in range(n + 1):
            assert int(em[k == kk].sum()) == math.comb(n, kk)


@pytest.mark.parametrize("n", [2, 5, 8, 10])
def test_column_counts_lemma6(n):
    """Lemma 6 (CS75): every y of length k has sum_{i<=n-k} C(n,i) length-n
    supersequences, so column y of W has that many nonzeros."""
    E = bdc.emb_dense(n)
    k = bdc.output_lengths(n)
    col_nnz = (E > 0).sum(axis=0)
    for r in range(E.shape[1]):
        kk = int(k[r])
        assert col_nnz[r] == sum(math.comb(n, i) for i in range(n - kk + 1))


@pytest.mark.parametrize("n", [1, 2, 4, 7, 10, 12])
def test_total_nonzeros(oracle_native, n):
    """nnz(W) = sum_k 2^k sum_{i<=n-k} C(n,i) = 2*3^n - 2^n."""
    closed = 2 * 3 ** n - 2 ** n
    via_lemma6 = sum((1 << k) * sum(math.comb(n, i) for i in range(n - k + 1)) for k in range(n + 1))
    assert closed == via_lemma6
    if n <= 10:
        assert int((bdc.emb_dense(n) > 0).sum()) == closed
    assert oracle_native.CSR(n).nnz == closed


def count_table(x, n):
    """NextPos (Algorithm 3) and the Count recurrence of Section 4.1, written
    independently here: Count[i][t] = number of distinct length-t subsequences of
    x[i:n-1]."""
    xb = bits_of(x, n)
    nxt = [[n, n] for _ in range(n + 1)]
    for i in range(n - 1, -1, -1):
        nxt[i] = list(nxt[i + 1])
        nxt[i][xb[i]] = i
    cnt = [[0] * (n + 1) for _ in range(n + 1)]
    for i in range(n + 1):
        cnt[i][0] = 1
    for i in range(n - 1, -1, -1):
        for t in range(1, n + 1):
            j0, j1 = nxt[i]
            c = 0
            if j0 < n:
                c += cnt[j0 + 1][t - 1]
            if j1 < n:
                c += cnt[j1 + 1][t - 1]
            cnt[i][t] = c
    return cnt


@pytest.mark.parametrize("n", [3, 6, 9])
def test_row_nonzeros_equal_count_table(n):
    E = bdc.emb_dense(n)
    k = bdc.output_lengths(n)
    for x in range(1 << n):
        cnt = count_table(x, n)
        for kk in range(n + 1):
            assert int((E[x, k == kk] > 0).sum()) == cnt[0][kk]


@pytest.mark.parametrize("n", [4, 7])
def test_symmetry_complement_reversal(n):
    """eq. BDC-sym (Appendix A): P(g(y)|g(x)) = P(y|x) for g = cpl, rev and their
    composition."""
    E = bdc.emb_dense(n)
    for r in range(E.shape[1]):
        yb, k = bdc.unrank(r)
        for g in (lambda v, m: cpl(v, m), lambda v, m: rev(v, m), lambda v, m: rev(cpl(v, m), m)):
            r2 = bdc.rank(g(yb, k) if k else 0, k)
            for x in range(1 << n):
                assert E[x, r] == E[g(x, n), r2]


@pytest.mark.parametrize("n", [4, 9, 12])
def test_max_embedding_count(n):
    """max emb = C(n, floor(n/2)), reached at x = 0^n, y = 0^{floor(n/2)}."""
    rk, em = __import__("oracle.native", fromlist=["row"]).row(n, 0)
    assert int(em.max()) == math.comb(n, n // 2)
    assert int(rk[np.argmax(em)]) == bdc.rank(0, n // 2)
    if n <= 9:
        assert int(bdc.emb_dense(n).max()) == math.comb(n, n // 2)


# --------------------------------------------------------------------------
# Channel and one BA evaluation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [0.0, 0.2, 0.5, 0.95, 1.0])
def test_channel_rows_sum_to_one(d):
    W = bdc.channel_dense(6, d)
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-14)


def test_evaluate_matches_entropy_form():
    """I(X;Y) = sum_x X(x) D(x) against H(Y) - H(Y|X) with explicit sums."""
    n = 5
    W = bdc.channel_dense(n, 0.37)
    for seed in range(3):
        lp = inp.random_logp(n, seed=seed, spread=1.5)
        p = np.exp(bdc.normalise_logp(lp))
        ev = bdc.evaluate(W, lp)
        assert abs(ev.I - bdc.mutual_information_entropy_form(W, p)) < 1e-12
        assert ev.L >= ev.I - 1e-13  # Jensen: log E[e^D] >= E[D]
        assert ev.U >= ev.L - 1e-13


def test_uniform_output_closed_form():
    """At uniform X: r(y) = C(n,k) 2^-k for every y of length k."""
    n = 7
    W = bdc.channel_dense(n, 0.3)
    ev = bdc.evaluate(W, bdc.uniform_logp(n))
    M = -n * LN2
    q = ev.q_scaled * math.exp(M)
    w = bdc.length_weights(n, 0.3)[bdc.output_lengths(n)]
    assert np.allclose(q / w, bdc.r_uniform(n), rtol=1e-13)


def test_scaling_of_logp_is_irrelevant():
    n = 6
    W = bdc.channel_dense(n, 0.6)
    lp = inp.random_logp(n, seed=5)
    a = bdc.evaluate(W, lp)
    b = bdc.evaluate(W, lp + 123.0)
    assert abs(a.L - b.L) < 1e-12 and abs(a.U - b.U) < 1e-12
    assert np.allclose(a.D, b.D, atol=1e-12)


def test_product_law_closed_forms(oracle_native):
    """r(y) for a product input law: the oracle's recursion (Python and C) against
    the dense sum_x p(x) emb(y,x)."""
    n = 8
    pi1 = inp.product_bit_probs(n, seed=7)
    lp = inp.product_logp(n, pi1)
    E = bdc.emb_dense(n)
    r_dense = np.exp(lp) @ E
    ranks = np.arange(E.shape[1])
    r_c = oracle_native.product_r(n, pi1, ranks)
    assert np.allclose(r_c, r_dense, rtol=1e-12, atol=0)
    for r in [0, 1, 2, 17, 200, E.shape[1] - 1]:
        yb, k = bdc.unrank(r)
        assert abs(bdc.r_product(n, pi1, yb, k) - r_dense[r]) <= 1e-12 * r_dense[r]
    d = 0.7
    W = bdc.channel_dense(n, d, E)
    ev = bdc.evaluate(W, lp)
    xs = np.arange(1 << n, dtype=np.uint32)
    D_c = oracle_native.product_D(n, d, pi1, xs)
    assert np.allclose(D_c, ev.D, atol=1e-11)


# --------------------------------------------------------------------------
# Blahut-Arimoto and its bounds
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [0.0, 0.1, 0.5, 0.83, 1.0])
def test_capacity_n1_is_one_minus_d(d):
    vals = paper_values()
    W = bdc.channel_dense(1, d)
    res = bdc.ba(W, 1, tol_bits=1e-12, max_iters=10000)
    want = vals["C1_intercept"] + vals["C1_slope"] * d
    assert res.lower_bits <= want + 1e-12 <= res.upper_bits + 2e-12
    assert abs(res.lower_bits - want) < 1e-10


@pytest.mark.parametrize("n", [1, 3, 6])
def test_capacity_d0_is_n_and_d1_is_0(n):
    """d = 0: the channel is the identity on n bits, C_n(0) = n; d = 1: the output
    is always empty, C_n(1) = 0.  Uniform X is optimal in both, so BA stops at t=0."""
    r0 = bdc.ba(bdc.channel_dense(n, 0.0), n, 1e-12, 10)
    assert r0.iters == 0
    assert abs(r0.lower_bits - n) < 1e-12 and abs(r0.upper_bits - n) < 1e-12
    r1 = bdc.ba(bdc.channel_dense(n, 1.0), n, 1e-12, 10)
    assert abs(r1.lower_bits) < 1e-12 and abs(r1.upper_bits) < 1e-12


def mi_symmetric_n2(d, a):
    """I(X;Y) for n = 2 with X(00) = X(11) = a, X(01) = X(10) = 1/2 - a, from the
    hand-written channel of tests/golden/emb_n2.txt (entropy form)."""
    E = {0: [1, 2, 0, 1, 0, 0, 0], 1: [1, 1, 1, 0, 1, 0, 0],
         2: [1, 1, 1, 0, 0, 1, 0], 3: [1, 0, 2, 0, 0, 0, 1]}
    k = [0, 1, 1, 2, 2, 2, 2]
    w = [d * d, d * (1 - d), (1 - d) * (1 - d)]
    p = {0: a, 1: 0.5 - a, 2: 0.5 - a, 3: a}
    W = {x: [E[x][r] * w[k[r]] for r in range(7)] for x in range(4)}
    q = [sum(p[x] * W[x][r] for x in range(4)) for r in range(7)]
    hy = -sum(v * math.log2(v) for v in q if v > 0)
    hyx = -sum(p[x] * sum(v * math.log2(v) for v in W[x] if v > 0) for x in range(4))
    return hy - hyx


@pytest.mark.parametrize("d", [0.2, 0.5, 0.8])
def test_n2_capacity_by_direct_maximisation(d):
    """C_2(d) by golden-section search over the symmetric family (the optimum is
    cpl/rev invariant, Theorem 4), independent of BA."""
    lo, hi = 0.0, 0.5
    g = (math.sqrt(5) - 1) / 2
    for _ in range(200):
        a1 = hi - g * (hi - lo)
        a2 = lo + g * (hi - lo)
        if mi_symmetric_n2(d, a1) < mi_symmetric_n2(d, a2):
            lo = a1
        else:
            hi = a2
    cap = mi_symmetric_n2(d, 0.5 * (lo + hi))
    res = bdc.ba(bdc.channel_dense(2, d), 2, tol_bits=1e-11, max_iters=100000)
    assert res.lower_bits - 1e-10 <= cap <= res.upper_bits + 1e-10
    assert abs(res.lower_bits - cap) < 1e-9


def test_ba_monotone_and_bracketing():
    """Theorem 1: I(X^{(t)};Y) is non-decreasing; every lower bound is below every
    upper bound (both bracket C)."""
    n = 6
    W = bdc.channel_dense(n, 0.55)
    res = bdc.ba(W, n, tol_bits=1e-9, max_iters=400, keep_history=True)
    L = np.array([h[0] for h in res.history])
    U = np.array([h[1] for h in res.history])
    I = np.array([h[2] for h in res.history])
    assert np.all(np.diff(I) >= -1e-13)
    assert L.max() <= U.min() + 1e-12
    assert np.all(I <= L + 1e-13)


def test_stopping_quantity_is_max_log_ratio():
    """max_x log(X^{(t+1)}/X^{(t)}) (Section 2.3 stopping rule) equals U - L."""
    n = 5
    W = bdc.channel_dense(n, 0.42)
    lp = bdc.normalise_logp(inp.random_logp(n, seed=9, spread=1.0))
    ev = bdc.evaluate(W, lp)
    nxt = bdc.ba_update(lp, ev)
    assert abs(np.max(nxt - lp) - (ev.U - ev.L)) < 1e-12
    assert abs(math.log(np.exp(nxt).sum())) < 1e-12


def test_symmetry_of_iterates_theorem4():
    """Theorem 4: from uniform X^{(0)}, X^{(t)}(g(x)) = X^{(t)}(x) at every t."""
    n = 6
    W = bdc.channel_dense(n, 0.7)
    lp = bdc.uniform_logp(n)
    xs = np.arange(1 << n)
    gc = np.array([cpl(x, n) for x in xs])
    gr = np.array([rev(x, n) for x in xs])
    for _ in range(30):
        lp = bdc.ba_update(lp, bdc.evaluate(W, lp))
        assert np.max(np.abs(lp[gc] - lp)) < 1e-12
        assert np.max(np.abs(lp[gr] - lp)) < 1e-12


def converged(n, d, tol=1e-8, iters=200000):
    return bdc.ba(bdc.channel_dense(n, d), n, tol_bits=tol, max_iters=iters)


def test_subadditivity_and_erasure_bound():
    """C_{m+n} <= C_m + C_n (the subadditivity behind Lemma 1) and
    C_n(d) <= n C_1(d) = n (1-d)."""
    d = 0.5
    c2, c4, c6 = converged(2, d), converged(4, d), converged(6, d)
    assert c6.lower_bits <= c4.upper_bits + c2.upper_bits + 1e-9
    assert c4.lower_bits <= 2 * c2.upper_bits + 1e-9
    for c, n in ((c2, 2), (c4, 4), (c6, 6)):
        assert c.lower_bits <= n * (1 - d) + 1e-12


def test_monotone_in_deletion_probability():
    """BDC_{d2} is BDC_{d1} followed by an independent BDC, so C_n(d) is
    non-increasing in d (data processing)."""
    n = 5
    prev = None
    for d in [0.3, 0.45, 0.6, 0.75, 0.9]:
        c = converged(n, d, tol=1e-9)
        if prev is not None:
            assert c.lower_bits <= prev.upper_bits + 1e-12
        prev = c


def test_floored_iterates_keep_valid_bounds():
    """The floored update (ba_update with floor_nats) keeps every log p within
    floor_nats of the maximum, equals the plain update wherever the floor does not
    bind, and the Blahut bounds of its iterates stay valid: every lower bound seen,
    floored or not, is below every upper bound seen (each brackets the same
    capacity)."""
    n, d = 8, 0.8
    W = bdc.channel_dense(n, d)
    lp = bdc.uniform_logp(n)
    plain = bdc.uniform_logp(n)
    Ls, Us = [], []
    floored_seen = 0
    for t in range(1500):
        ev = bdc.evaluate(W, lp)
        Ls.append(ev.L)
        Us.append(ev.U)
        nxt = bdc.ba_update(lp, ev, floor_nats=50.0)
        free = bdc.normalise_logp(lp) + ev.D - ev.L
        assert np.all(nxt >= nxt.max() - 50.0 - 1e-12)
        at_floor = free < free.max() - 50.0
        assert np.array_equal(nxt[~at_floor], free[~at_floor])
        floored_seen = max(floored_seen, int(at_floor.sum()))
        lp = nxt
        if t < 300:
            evp = bdc.evaluate(W, plain)
            Ls.append(evp.L)
            Us.append(evp.U)
            plain = bdc.ba_update(plain, evp)
    assert floored_seen > 10
    assert max(Ls) <= min(Us) + 1e-12
    assert min(Us) - max(Ls) < 1e-3


def test_certify_floor_keeps_bounds_finite():
    n = 5
    W = bdc.channel_dense(n, 0.6)
    lp = bdc.uniform_logp(n)
    lp[3] = -1e6
    L, U = bdc.certify(W, lp)
    assert math.isfinite(L) and math.isfinite(U) and L <= U


# --------------------------------------------------------------------------
# Gradients and mirror ascent
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,d", [(3, 0.4), (5, 0.8)])
def test_gradients_against_central_differences(n, d):
    E = bdc.emb_dense(n)
    theta = inp.theta_normal(n, seed=0, sigma=0.5)
    I, g_theta, g_d = bdc.info_and_grads(n, d, theta, E)
    assert abs(I - bdc.info_bits(n, d, theta, E)) < 1e-13
    h = 1e-6
    for j in range(1 << n):
        e = np.zeros_like(theta)
        e[j] = h
        fd = (bdc.info_bits(n, d, theta + e, E) - bdc.info_bits(n, d, theta - e, E)) / (2 * h)
        assert abs(fd - g_theta[j]) <= 1e-8 + 1e-5 * abs(g_theta[j])
    fd_d = (bdc.info_bits(n, d + h, theta, E) - bdc.info_bits(n, d - h, theta, E)) / (2 * h)
    assert abs(fd_d - g_d) <= 1e-8 + 1e-5 * abs(g_d)
    assert abs(g_theta.sum()) < 1e-12  # softmax gradients sum to zero


def test_mirror_ascent_with_unit_step_is_ba():
    n = 5
    d = 0.65
    E = bdc.emb_dense(n)
    W = bdc.channel_dense(n, d, E)
    theta = inp.theta_normal(n, seed=0, sigma=0.3)
    th = bdc.mirror_ascent(n, d, theta, 1.0, 25, E)
    lp = bdc.ba_iterate(W, bdc.normalise_logp(theta), 25)
    assert np.allclose(bdc.normalise_logp(th), lp, atol=1e-12)


def test_mirror_ascent_step_derivative_is_variance_of_D():
    """One mirror-ascent step p_eta ~ p e^{eta D} moves I at eta = 0 with slope
    dI/deta = sum_x (dI/dp(x)) p(x) (D(x) - I) = Var_p(D) (nats), since
    dI/dp(x) = D(x) - 1 and sum_x p (D - I) = 0.  A step that rescales theta or the
    normalised log p by eta, or drops the current theta, has another slope.  Small
    steps increase I."""
    n, d = 5, 0.65
    E = bdc.emb_dense(n)
    W = bdc.channel_dense(n, d, E)
    theta = inp.theta_normal(n, seed=3, sigma=0.7)
    ev = bdc.evaluate(W, bdc.normalise_logp(theta))
    p = bdc.softmax(theta)
    var = float(p @ (ev.D - ev.I) ** 2)
    assert var > 1e-3

    def I_after(eta):
        return bdc.info_bits(n, d, bdc.mirror_ascent(n, d, theta, eta, 1, E), E) * LN2

    assert abs(I_after(0.0) - ev.I) < 1e-13
    h = 1e-5
    slope = (I_after(h) - I_after(-h)) / (2 * h)
    assert abs(slope - var) < 1e-8
    # a second step from the first: its slope is the variance at the new law
    th1 = bdc.mirror_ascent(n, d, theta, 0.5, 1, E)
    ev1 = bdc.evaluate(W, bdc.normalise_logp(th1))
    p1 = bdc.softmax(th1)
    var1 = float(p1 @ (ev1.D - ev1.I) ** 2)
    th2 = lambda eta: bdc.info_bits(n, d, th1 + eta * ev1.D, E) * LN2
    assert abs((th2(h) - th2(-h)) / (2 * h) - var1) < 1e-8
    assert np.allclose(bdc.normalise_logp(bdc.mirror_ascent(n, d, theta, 0.5, 2, E)),
                       bdc.normalise_logp(th1 + 0.5 * ev1.D), atol=1e-12)
    for eta in (0.05, 0.2, 0.5):
        assert I_after(eta) > ev.I


# --------------------------------------------------------------------------
# The certify-only tier: per-row generator and full-size evaluation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 8, 10])
def test_row_generator_every_row_matches_brute_force(oracle_native, n):
    for x in range(1 << n):
        a = oracle_native.row(n, x)
        b = oracle_native.row_dp(n, x)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (n, x)


def test_row_generator_matches_brute_force_n20(oracle_native):
    """256 seeded rows of the n = 20 channel, including 0^n, 1^n and both alternating
    strings, bit-exact against the subset definition."""
    n = 20
    xs = inp.sample_rows(n, 256, seed=31)
    full = (1 << n) - 1
    alt = int("01" * 10, 2)
    for must in (0, full, alt, full ^ alt):
        assert must in xs
    assert len(xs) >= 256
    A = oracle_native.rows(n, xs, cap=30000)
    B = oracle_native.rows_dp(n, xs, cap=30000)
    for x, a, b in zip(xs, A, B):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), x


def test_certify_matches_csr_evaluation(oracle_native):
    """bdc_certify against the CSR evaluation (itself pinned to the dense channel),
    three instances at once: two BDC_d and one exact channel BDC_{n,k}, random
    laws, with and without the 700-nat floor."""
    n = 12
    csr = oracle_native.CSR(n)
    ds = [0.64, 0.9]
    wexact = np.zeros(n + 1)
    wexact[5] = 1.0 / math.comb(n, 5)
    weights = [bdc.length_weights(n, d) for d in ds] + [wexact]
    lps = [inp.random_logp(n, seed=40 + i, spread=2.0 + 60.0 * (i == 1)) for i in range(3)]
    for floor in (700.0, 0.0):
        out = oracle_native.certify(n, weights, lps, floor_nats=floor, want_r=True)
        for i in range(2):
            D, L, U, I, q = csr.evaluate(ds[i], lps[i], floor_nats=floor, want_q=True)
            assert np.allclose(out["D"][i], D, atol=1e-11, rtol=0)
            assert abs(out["L"][i] - L) < 1e-11 and abs(out["U"][i] - U) < 1e-11 and abs(out["I"][i] - I) < 1e-11
            w = bdc.length_weights(n, ds[i])[bdc.output_lengths(n)]
            assert np.allclose(out["r"][i] * w, q, rtol=1e-12, atol=0)
        ex = bdc.evaluate(bdc.channel_dense_exact(n, 5), bdc.floor_logp(bdc.normalise_logp(lps[2]),
                                                                        floor or None))
        assert np.allclose(out["D"][2], ex.D, atol=1e-11, rtol=0)
        assert abs(out["L"][2] - ex.L) < 1e-11 and abs(out["U"][2] - ex.U) < 1e-11
    assert out["stats"] == {"nnz": 2 * 3 ** n - 2 ** n, "bad_rows": 0, "min_row_nnz": n + 1,
                            "max_row_nnz": out["stats"]["max_row_nnz"], "max_emb": math.comb(n, n // 2)}


@pytest.mark.slow
def test_certify_n20_product_laws(oracle_native):
    """The certify-only tier over every row of the n = 20 channel at product laws,
    against their closed forms: r(y) at 4000 seeded outputs and D(x) at 64 seeded
    rows; and the whole-matrix count invariants: 2*3^n - 2^n nonzeros, every row's
    length sums equal to C(n,k), minimum row nnz n+1, maximum emb C(n, n/2)."""
    n = 20
    ds = [0.64, 0.95]
    pis = [inp.product_bit_probs(n, seed=50 + i) for i in range(2)]
    out = oracle_native.certify(n, [bdc.length_weights(n, d) for d in ds],
                                [inp.product_logp(n, pi) for pi in pis], want_r=True)
    st = out["stats"]
    assert st["nnz"] == 2 * 3 ** n - 2 ** n and st["bad_rows"] == 0
    assert st["min_row_nnz"] == n + 1 and st["max_emb"] == math.comb(n, n // 2)
    ranks = inp.sample_outputs(n, 4000, seed=51)
    xs = inp.sample_rows(n, 64, seed=52)
    for i in range(2):
        want_r = oracle_native.product_r(n, pis[i], ranks)
        got_r = out["r"][i][ranks] * math.exp(out["M"][i])
        assert np.allclose(got_r, want_r, rtol=1e-11, atol=0)
        assert np.allclose(out["D"][i][xs], oracle_native.product_D(n, ds[i], pis[i], xs), atol=1e-10, rtol=0)
        assert out["L"][i] <= out["U"][i]


# --------------------------------------------------------------------------
# The C CSR implementation against the numpy dense one
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,d", [(6, 0.5), (9, 0.72)])
def test_csr_matches_dense(oracle_native, n, d):
    W = bdc.channel_dense(n, d)
    csr = oracle_native.CSR(n)
    lp = inp.random_logp(n, seed=n, spread=2.0)
    ev = bdc.evaluate(W, lp)
    D, L, U, I, q = csr.evaluate(d, lp, want_q=True)
    assert np.allclose(D, ev.D, atol=1e-12)
    assert abs(L - ev.L) < 1e-12 and abs(U - ev.U) < 1e-12 and abs(I - ev.I) < 1e-12
    assert np.allclose(q, ev.q_scaled, rtol=1e-12, atol=1e-300)
    a = csr.iterate(d, lp, 20)
    b = bdc.ba_iterate(W, bdc.normalise_logp(lp), 20)
    assert np.allclose(bdc.normalise_logp(a), b, atol=1e-11)


def exact_capacity(n, k, tol=1e-10):
    return bdc.ba(bdc.channel_dense_exact(n, k), n, tol_bits=tol, max_iters=200000)


def test_exact_channel_paper_values():
    """Section 6 states C_{2,1} = 1 and C_{2,2} = 2; Table 1 gives C_{29,1} = 1.0000
    and C_{29,29} = 29.0000, i.e. C_{n,1} = 1 (one output bit, achieved by 0^n and
    1^n) and C_{n,n} = n (no deletion).  C_{n,0} = 0 (the output is always empty)."""
    vals = paper_values()
    assert abs(exact_capacity(2, 1).lower_bits - vals["C_2_1"]) < 1e-9
    assert abs(exact_capacity(2, 2).lower_bits - vals["C_2_2"]) < 1e-9
    for n in (3, 5, 7):
        assert abs(exact_capacity(n, 1).lower_bits - vals["C_29_1"]) < 1e-9
        assert abs(exact_capacity(n, n).upper_bits - n * vals["C_29_29"] / 29.0) < 1e-9
        assert abs(exact_capacity(n, 0).upper_bits) < 1e-12
    for n in range(1, 8):
        W = bdc.channel_dense_exact(n, min(n, 3))
        assert np.allclose(W.sum(axis=1), 1.0, atol=1e-14)


def test_exact_channel_lemma_2():
    """Lemma 2 (C_n(d) <= sum_k pi_k C_{n,k}) holds between independently computed
    brackets: the BDC_d lower bound against the exact channels' upper bounds."""
    n = 6
    U = [exact_capacity(n, k, 1e-9).upper_bits for k in range(n + 1)]
    for d in (0.2, 0.5, 0.8):
        Cn = bdc.ba(bdc.channel_dense(n, d), n, tol_bits=1e-9, max_iters=200000)
        assert Cn.lower_bits <= bdc.lemma2_bound(n, d, U) + 1e-9


def test_sample_sweeps_match_dense(oracle_native):
    """The bounded-sample sweeps (used for the CPU baseline) against the dense
    evaluation: q restricted to the sampled rows and D at those rows."""
    n, d = 7, 0.55
    W = bdc.channel_dense(n, d)
    lp = bdc.normalise_logp(inp.random_logp(n, seed=8))
    p = np.exp(lp)
    q_full = p @ W
    xs = inp.sample_rows(n, 20, seed=3)
    q_part, D, tot = oracle_native.sample_sweeps(n, d, p, xs, q_full)
    assert np.allclose(q_part, p[xs] @ W[xs], rtol=1e-13, atol=1e-300)
    ev = bdc.evaluate(W, lp)
    assert np.allclose(D, ev.D[xs], atol=1e-12)
    assert tot == int((W[xs] > 0).sum())


# ---------------------------------------------------------------------------
# supersequence enumeration (Section 5)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 7])
def test_subset_unrank_lists_every_subset_once_in_order(n):
    """Algorithm 5: j -> the j-th w-subset is a bijection onto the w-subsets, and
    the order puts subsets containing the smaller element first (lexicographic
    order of the characteristic vectors, largest first)."""
    for w in range(n + 1):
        subs = [tuple(bdc.subset_unrank(n, w, j)) for j in range(math.comb(n, w))]
        assert len(set(subs)) == math.comb(n, w)
        assert all(len(s) == w and all(0 <= t < n for t in s) for s in subs)
        vec = [sum(1 << (n - 1 - t) for t in s) for s in subs]
        assert vec == sorted(vec, reverse=True)


@pytest.mark.parametrize("n", [1, 2, 4, 6, 8])
def test_supersequence_enumeration_is_a_bijection(n):
    """Section 5.2 with Lemma 7: for every y the position sets S with |S| <= n - k
    name its supersequences one-to-one, and index i = sum_{j<w} C(n,j) + (rank of S
    among the w-subsets, Section 5.1) lists them all."""
    for k in range(n + 1):
        assert bdc.supersequence_count(n, k) == sum(math.comb(n, i) for i in range(n - k + 1))
        for yb in range(1 << k):
            y = [(yb >> (k - 1 - q)) & 1 for q in range(k)]
            sup = [x for x in range(1 << n) if bdc.emb_brute(y, bdc.string_bits(x, n)) > 0]
            assert len(sup) == bdc.supersequence_count(n, k)
            xs = [bdc.supersequence(i, n, y) for i in range(bdc.supersequence_count(n, k))]
            assert sorted(xs) == sup, (n, yb, k)
            i = 0
            for w in range(n - k + 1):
                for j in range(math.comb(n, w)):
                    assert bdc.supersequence_key(xs[i], n, y) == tuple(bdc.subset_unrank(n, w, j))
                    i += 1


def test_supersequence_key_examples():
    """Hand-checked keys: y = 01 in x = 1001 is embedded at positions 1, 3 (position 0
    skipped, position 2 skipped); in x = 0111 at 0, 1 with tail 11 = y's last symbol;
    in x = 0110 at 0, 1 with position 3 differing from the last symbol 1."""
    assert bdc.supersequence_key(0b1001, 4, [0, 1]) == (0, 2)
    assert bdc.supersequence_key(0b0111, 4, [0, 1]) == ()
    assert bdc.supersequence_key(0b0110, 4, [0, 1]) == (3,)
    assert bdc.supersequence_key(0b101, 3, []) == (0, 2)


def test_printed_supersequence_rule_is_not_one_to_one():
    """Section 5.2 as printed fills the positions after the embedding with
    1 - y_{k-1} in S and 0 outside S.  For a y ending in 1 both are 0, so it only
    reaches the supersequences whose tail after the leftmost embedding is all 0,
    fewer than the sum_{i<=n-k} C(n,i) of Lemma 7: it repeats strings.  For a y
    ending in 0 any tail is reachable and the printed rule and the reading used
    here coincide."""
    n = 3
    for y, repeats in (([1], True), ([0], False), ([0, 1], True), ([1, 0], False)):
        sup = [x for x in range(1 << n) if bdc.emb_brute(y, bdc.string_bits(x, n)) > 0]
        reach = []
        for x in sup:
            xb = bdc.string_bits(x, n)
            r, pos = 0, 0
            while r < len(y):
                r += xb[pos] == y[r]
                pos += 1
            if y[-1] == 0 or all(b == 0 for b in xb[pos:]):
                reach.append(x)
        assert (len(reach) < bdc.supersequence_count(n, len(y))) == repeats


@pytest.mark.parametrize("n", [3, 6])
def test_pull_sum_matches_push(n):
    """r(y) summed over supersequences equals column y of E^T p (dense)."""
    lp = inp.random_logp(n, seed=70 + n, spread=2.0)
    E = bdc.emb_dense(n)
    r = np.exp(lp) @ E
    for R in range((2 << n) - 1):
        yb, k = bdc.unrank(R)
        assert abs(bdc.r_pull(n, lp, yb, k) - r[R]) <= 1e-12 * max(1.0, abs(r[R]))


# ---------------------------------------------------------------------------
# orbit-reduced output law (Appendix A)
# ---------------------------------------------------------------------------

def test_orbit_examples():
    """Hand-checked orbits: 0110 is its own complement-reversal image; 0011 maps to
    1100 (complement) and 1100 (reversal); 0001 has four members."""
    assert bdc.orbit(0b0110, 4) == {0b0110, 0b1001}
    assert bdc.orbit(0b0011, 4) == {0b0011, 0b1100}
    assert bdc.orbit(0b0001, 4) == {0b0001, 0b1110, 0b1000, 0b0111}
    assert bdc.orbit(0, 0) == {0}
    assert bdc.orbit_rep(0b1110, 4) == 0b0001


@pytest.mark.parametrize("n", [3, 5, 6])
def test_orbit_output_law_equals_full_sum_for_invariant_laws(n):
    """Algorithm 7 gives r = E^T p exactly (to rounding) for laws invariant under
    complement and reversal: the uniform law, a random invariant law and a BA
    iterate from the uniform law (Theorem 4); it does not for a law that is not
    invariant (the reduction relies on that invariance)."""
    E = bdc.emb_dense(n)
    W = bdc.channel_dense(n, 0.7, E)
    rng = np.random.default_rng(60 + n)
    inv = np.zeros(1 << n)
    for x in range(1 << n):
        rep = bdc.orbit_rep(x, n)
        if rep == x:
            inv[[y for y in bdc.orbit(x, n)]] = rng.normal(0, 1.5)
    it = bdc.ba_iterate(W, bdc.uniform_logp(n), 7)
    for lp in (bdc.uniform_logp(n), inv, it):
        full = np.exp(bdc.normalise_logp(lp)) @ E
        assert np.allclose(bdc.r_orbits(n, lp), full, rtol=1e-13, atol=0)
    bad = inp.random_logp(n, seed=61, spread=2.0)
    assert not np.allclose(bdc.r_orbits(n, bad), np.exp(bdc.normalise_logp(bad)) @ E, rtol=1e-6)
