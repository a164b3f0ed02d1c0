"""Plain FP64 numpy oracle (test infrastructure only; see ``oracle/__init__``).

Conventions
-----------
* Strings are indexed from 0 (paper, Section 2.1).  An input x in {0,1}^n is the
  integer sum_i x_i 2^(n-1-i): x_0 is the most significant bit, so lexicographic
  order is numeric order.
* An output y of length k has rank (2^k - 1) + sum_i y_i 2^(k-1-i); the ranks of
  all outputs of length <= n are 0 .. 2^(n+1)-2 (empty string = rank 0).
* Internal arithmetic is in nats.  Bounds, rates and gradients are reported in
  bits (the paper's logarithms are base 2, Section 2.1) by dividing by ln 2.

Every function below names the passage of the paper it writes out.
"""
from __future__ import annotations

import functools
import itertools
import math
from dataclasses import dataclass

import numpy as np

LN2 = math.log(2.0)
DENSE_N_MAX = 12


def rank(bits: int, k: int) -> int:
    """Output rank of the length-k string whose bits, read as an integer with y_0
    most significant, equal ``bits``."""
    return (1 << k) - 1 + bits


def unrank(r: int) -> tuple[int, int]:
    """Inverse of :func:`rank`: returns (bits, k)."""
    k = (r + 1).bit_length() - 1
    return r - ((1 << k) - 1), k


def string_bits(x: int, n: int) -> list[int]:
    return [(x >> (n - 1 - i)) & 1 for i in range(n)]


def emb_brute(y: list[int], x: list[int]) -> int:
    """Number of embeddings of y in x: index sets i_1 < ... < i_k with
    x_{i_j} = y_j (Section 2.2, the numerator of P_{n,k}).  Pure-Python recursion
    over positions, for tiny inputs only."""
    k, n = len(y), len(x)
    if k == 0:
        return 1
    if n < k:
        return 0
    total = emb_brute(y, x[1:])  # x_0 not used
    if x[0] == y[0]:
        total += emb_brute(y[1:], x[1:])  # x_0 matched to y_0
    return total


def emb_dense(n: int) -> np.ndarray:
    """Matrix E[x, rank(y)] = emb(y, x) for all x in {0,1}^n and |y| <= n.

    Definition (Section 2.2): the count of position subsets S of {0..n-1} whose
    restriction x_S equals y.  Written out literally: for every subset S (as a
    bitmask over string positions) and every x, extract y = x_S and add one.
    int64, shape (2^n, 2^(n+1)-1); n <= DENSE_N_MAX."""
    if not 0 <= n <= DENSE_N_MAX:
        raise ValueError("dense counts need 0 <= n <= %d" % DENSE_N_MAX)
    xs = np.arange(1 << n, dtype=np.int64)
    E = np.zeros((1 << n, (1 << (n + 1)) - 1), dtype=np.int64)
    for S in range(1 << n):
        y = np.zeros_like(xs)
        k = 0
        for i in range(n):  # positions in increasing order
            if (S >> (n - 1 - i)) & 1:
                y = (y << 1) | ((xs >> (n - 1 - i)) & 1)
                k += 1
        E[xs, (1 << k) - 1 + y] += 1
    return E


def output_lengths(n: int) -> np.ndarray:
    """Length k of the output with each rank, shape (2^(n+1)-1,)."""
    r = np.arange((1 << (n + 1)) - 1, dtype=np.int64)
    return np.floor(np.log2(r + 1)).astype(np.int64)


def length_weights(n: int, d: float) -> np.ndarray:
    """w_k = d^(n-k) (1-d)^k, k = 0..n, with 0^0 = 1: the probability of one
    particular set of n-k deletions in BDC_d (Section 2.2, each bit deleted
    independently with probability d)."""
    return np.array([(d ** (n - k)) * ((1.0 - d) ** k) for k in range(n + 1)])


def channel_dense(n: int, d: float, E: np.ndarray | None = None) -> np.ndarray:
    """W[x, rank(y)] = emb(y, x) d^(n-|y|) (1-d)^|y|: the law of BDC_d on
    n-bit inputs (Section 2.2, the finite-length DMC whose capacity is C_n(d))."""
    if E is None:
        E = emb_dense(n)
    return E * length_weights(n, d)[output_lengths(n)][None, :]


def channel_dense_exact(n: int, k: int, E: np.ndarray | None = None) -> np.ndarray:
    """W[x, rank(y)] = emb(y, x) / C(n, k) for |y| = k, 0 otherwise: the exact
    deletion channel BDC_{n,k} of Section 2.2 (a uniformly random set of n-k
    positions is deleted), whose capacity is C_{n,k}."""
    if E is None:
        E = emb_dense(n)
    w = np.zeros(n + 1)
    w[k] = 1.0 / math.comb(n, k)
    return E * w[output_lengths(n)][None, :]


def lemma2_bound(n: int, d: float, c_nk) -> float:
    """Lemma 2: C_n(d) <= sum_k C(n,k) d^(n-k) (1-d)^k C_{n,k}; c_nk[k] for k = 0..n
    (the k = 0 term is C_{n,0} = 0)."""
    w = length_weights(n, d)
    return float(sum(math.comb(n, k) * w[k] * c_nk[k] for k in range(n + 1)))


# ---------------------------------------------------------------------------
# One Blahut-Arimoto iteration, in the order of Section 2.3 (and Algorithm 1).
# Probabilities are carried as logs; the paper itself evaluates log W^{(t)} for
# numerical stability (Section 3).
# ---------------------------------------------------------------------------

def floor_logp(lp: np.ndarray, floor_nats: float | None) -> np.ndarray:
    """Optional floor relative to the largest entry: max(lp, max(lp) - floor).
    The certified evaluation uses floor = 700 nats so that every input keeps a
    representable probability (reading of an edge the paper does not treat)."""
    if floor_nats is None:
        return lp
    return np.maximum(lp, lp.max() - floor_nats)


def normalise_logp(lp: np.ndarray) -> np.ndarray:
    """Subtract log sum exp so that exp(lp) sums to one."""
    m = lp.max()
    return lp - (m + math.log(np.exp(lp - m).sum()))


@dataclass
class Eval:
    """Quantities of one BA iteration at input distribution X = exp(lp)."""
    q_scaled: np.ndarray  # output distribution Y^{(t)} times exp(-max lp)
    D: np.ndarray         # D(x) = sum_y P(y|x) log(P(y|x)/Y(y)), nats
    L: float              # log sum_x X(x) e^{D(x)}, nats (Blahut lower bound)
    U: float              # max_x D(x), nats (Blahut upper bound)
    I: float              # I(X;Y) = sum_x X(x) D(x), nats


def evaluate(W: np.ndarray, lp: np.ndarray) -> Eval:
    """Steps 1 and 2(a) of Section 2.3 at X = exp(lp) (lp normalised or not: the
    formulas below renormalise).

    Y(y) = sum_x X(x) P(y|x); log W(x) = log X(x) + D(x) with
    D(x) = sum_y P(y|x) log(P(y|x)/Y(y)) (0 log 0 = 0).  The stopping quantity
    max_x log(X^{(t+1)}(x)/X^{(t)}(x)) equals U - L with U = max_x D(x) and
    L = log sum_x X(x) e^{D(x)}; by Blahut's and Arimoto's bounds L <= C <= U."""
    lp = normalise_logp(lp)
    M = lp.max()
    p_scaled = np.exp(lp - M)               # X(x) e^{-M}
    q_scaled = p_scaled @ W                 # Y(y) e^{-M}
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(W > 0, W / q_scaled[None, :], 1.0)
        D = np.where(W > 0, W * np.log(ratio), 0.0).sum(axis=1) - M * W.sum(axis=1)
    a = lp + D
    am = a.max()
    L = float(am + math.log(np.exp(a - am).sum()))
    U = float(D.max())
    I = float(np.dot(np.exp(lp), D))
    return Eval(q_scaled=q_scaled, D=D, L=L, U=U, I=I)


def ba_update(lp: np.ndarray, ev: Eval, floor_nats: float | None = None) -> np.ndarray:
    """Step 2(b) of Section 2.3: X^{(t+1)} = W^{(t)} / sum W^{(t)}, i.e.
    log X^{(t+1)} = log X^{(t)} + D - L.  With floor_nats, the new log law is then
    raised to at least its maximum minus floor_nats (reading: the paper leaves
    inputs whose probability decays to zero untreated; the floor keeps every input
    representable and the Blahut bounds of the floored law remain valid)."""
    return floor_logp(normalise_logp(lp) + ev.D - ev.L, floor_nats)


def uniform_logp(n: int) -> np.ndarray:
    """X^{(0)} uniform on {0,1}^n (Section 2.3)."""
    return np.full(1 << n, -n * LN2)


@dataclass
class BAResult:
    lower_bits: float
    upper_bits: float
    rate_bits: float
    iters: int
    lp: np.ndarray
    history: list | None = None


def ba(W: np.ndarray, n: int, tol_bits: float, max_iters: int,
       lp0: np.ndarray | None = None, keep_history: bool = False) -> BAResult:
    """The BAA of Section 2.3 with its stopping rule: iterate until
    max_x log(X^{(t+1)}/X^{(t)}) = U - L < tol (bits), or ``max_iters`` updates.

    Reported values are those of the last evaluated iterate X^{(t)}."""
    lp = uniform_logp(n) if lp0 is None else normalise_logp(np.asarray(lp0, float))
    hist = [] if keep_history else None
    t = 0
    while True:
        ev = evaluate(W, lp)
        if hist is not None:
            hist.append((ev.L / LN2, ev.U / LN2, ev.I / LN2))
        if (ev.U - ev.L) / LN2 < tol_bits or t >= max_iters:
            return BAResult(ev.L / LN2, ev.U / LN2, ev.I / LN2, t, lp, hist)
        lp = ba_update(lp, ev)
        t += 1


def ba_iterate(W: np.ndarray, lp: np.ndarray, iters: int, floor_nats: float | None = None) -> np.ndarray:
    """``iters`` BA updates from lp (no stopping test), optionally floored as in
    :func:`ba_update`."""
    for _ in range(iters):
        lp = ba_update(lp, evaluate(W, lp), floor_nats)
    return normalise_logp(lp)


def certify(W: np.ndarray, lp: np.ndarray, floor_nats: float = 700.0) -> tuple[float, float]:
    """FP64 certification at any input distribution: (L, U) in bits after the
    700-nat floor and renormalisation.  Both are valid bounds on C_n(d) for every
    full-support X (Blahut 1972)."""
    ev = evaluate(W, floor_logp(normalise_logp(lp), floor_nats))
    return ev.L / LN2, ev.U / LN2


# ---------------------------------------------------------------------------
# Mutual information and its derivatives (the differentiable form of the BA
# objective used for mirror ascent).
# ---------------------------------------------------------------------------

def softmax(theta: np.ndarray) -> np.ndarray:
    z = theta - theta.max()
    e = np.exp(z)
    return e / e.sum()


def mutual_information_entropy_form(W: np.ndarray, p: np.ndarray) -> float:
    """I(X;Y) = H(Y) - H(Y|X) in nats, computed from entropies with explicit
    sums; an independent formula used to pin :func:`evaluate`."""
    q = p @ W
    HY = -sum(float(v * math.log(v)) for v in q if v > 0)
    HYX = 0.0
    for xi in range(W.shape[0]):
        row = W[xi]
        HYX -= p[xi] * sum(float(v * math.log(v)) for v in row if v > 0)
    return HY - HYX


def length_scores(n: int, d: float) -> np.ndarray:
    """s_k = d/dd log w_k = (n-k)/d - k/(1-d) (needs 0 < d < 1)."""
    return np.array([(n - k) / d - k / (1.0 - d) for k in range(n + 1)])


def info_and_grads(n: int, d: float, theta: np.ndarray, E: np.ndarray | None = None):
    """I(p; d) for p = softmax(theta) in bits, with closed-form gradients:
    dI/dtheta = p (D - I) and dI/dd = sum_x p(x) sum_y s_k W log(W/q), both in
    bits.  (Derivation: dI/dp(x) = D(x) - 1 because sum_x' p(x') dD(x')/dp(x) =
    -sum_y W(y|x) = -1; and dW/dd = s_k W with sum_y s_k q(y) = sum_x p sum_y s_k W.)"""
    if E is None:
        E = emb_dense(n)
    W = channel_dense(n, d, E)
    p = softmax(theta)
    q = p @ W
    with np.errstate(divide="ignore", invalid="ignore"):
        logratio = np.where(W > 0, np.log(np.where(W > 0, W, 1.0) / q[None, :]), 0.0)
    D = (W * logratio).sum(axis=1)
    I = float(p @ D)
    s = length_scores(n, d)[output_lengths(n)]
    Dd = (W * s[None, :] * logratio).sum(axis=1)
    return I / LN2, p * (D - I) / LN2, float(p @ Dd) / LN2


def info_bits(n: int, d: float, theta: np.ndarray, E: np.ndarray | None = None) -> float:
    """I(p; d) in bits for p = softmax(theta) (value only)."""
    if E is None:
        E = emb_dense(n)
    W = channel_dense(n, d, E)
    p = softmax(theta)
    return evaluate(W, np.log(p)).I / LN2


def mirror_ascent(n: int, d: float, theta: np.ndarray, eta: float, steps: int,
                  E: np.ndarray | None = None) -> np.ndarray:
    """Entropic mirror ascent on I(p) over the simplex with p = softmax(theta):
    theta <- theta + eta * dI/dp (nats).  Constant shifts of dI/dp = D - 1 do not
    change softmax, so the step is theta <- theta + eta * D; eta = 1 is exactly
    the BA update of Section 2.3."""
    if E is None:
        E = emb_dense(n)
    W = channel_dense(n, d, E)
    th = np.array(theta, dtype=float)
    for _ in range(steps):
        ev = evaluate(W, th - th.max())
        th = th + eta * ev.D
        th = th - th.max()
    return th


# ---------------------------------------------------------------------------
# Supersequence enumeration (Section 5): the pull form of step 1 of Section 2.3,
# r(y) = sum over the length-n supersequences x of y of p(x) emb(y, x).
# ---------------------------------------------------------------------------

def binom_le(n: int, t: int) -> int:
    """sum_{j <= t} C(n, j), 0 for t < 0 (Section 5.1's notation)."""
    return sum(math.comb(n, j) for j in range(0, t + 1)) if t >= 0 else 0


def subset_unrank(n: int, w: int, j: int) -> list[int]:
    """The j-th w-subset of {0..n-1} in the order Section 5.1 enumerates them:
    lexicographic order of the increasing element lists (subsets holding the
    smaller element first), which is the order itertools.combinations yields."""
    assert 0 <= j < math.comb(n, w)
    return list(next(itertools.islice(itertools.combinations(range(n), w), j, None)))


def supersequence_key(x: int, n: int, y: list[int]) -> tuple[int, ...]:
    """The position set S that names the supersequence x of y in Section 5.2:
    the positions the leftmost embedding of y in x skips before it completes,
    together with the positions after it whose symbol differs from y's last
    symbol (for the empty y: the positions holding 1).  Returned sorted."""
    xb = string_bits(x, n)
    k = len(y)
    last = y[k - 1] if k > 0 else 0
    S, r = [], 0
    for pos in range(n):
        if r < k:
            if xb[pos] == y[r]:
                r += 1          # leftmost embedding: take the first match
            else:
                S.append(pos)   # skipped before the embedding completes
        elif xb[pos] != last:
            S.append(pos)       # tail position differing from y's last symbol
    assert r == k, "x is not a supersequence of y"
    return tuple(S)


@functools.lru_cache(maxsize=4096)
def _supersequences_in_order(n: int, y: tuple[int, ...]) -> tuple[int, ...]:
    sup = [x for x in range(1 << n) if emb_brute(list(y), string_bits(x, n)) > 0]
    return tuple(sorted(sup, key=lambda x: (len(supersequence_key(x, n, list(y))),
                                            supersequence_key(x, n, list(y)))))


def supersequence(i: int, n: int, y: list[int]) -> int:
    """The i-th length-n supersequence of y (Section 5.2), as an input index: the
    supersequences (found by brute force) ordered by their position set S from
    :func:`supersequence_key`, first by |S|, then as in :func:`subset_unrank`.
    Reading: Section 5.2 as printed writes 0 at the positions after the embedding
    outside S, which repeats strings when y ends in 1; naming the tail by the
    positions that differ from y's last symbol makes S -> x one-to-one."""
    return _supersequences_in_order(n, tuple(y))[i]


def supersequence_count(n: int, k: int) -> int:
    """Lemma 7 (Section 5): a length-k string has sum_{i <= n-k} C(n, i) length-n
    supersequences."""
    return binom_le(n, n - k)


def r_pull(n: int, lp: np.ndarray, y_bits: int, k: int) -> float:
    """r(y) = sum_x p(x) emb(y, x) with p = exp(lp), summed over the supersequences
    of y enumerated by Algorithm 6 (Section 5)."""
    y = [(y_bits >> (k - 1 - q)) & 1 for q in range(k)]
    tot = 0.0
    for i in range(supersequence_count(n, k)):
        x = supersequence(i, n, y)
        tot += math.exp(lp[x]) * emb_brute(y, string_bits(x, n))
    return tot


# ---------------------------------------------------------------------------
# Orbits under complement and reversal (Appendix A).
# ---------------------------------------------------------------------------

def orbit(bits: int, k: int) -> set[int]:
    """{y, cpl(y), rev(y), cpl(rev(y))} for the k-bit string y (Appendix A)."""
    full = (1 << k) - 1
    rv = int(format(bits, "0%db" % k)[::-1], 2) if k > 0 else 0
    return {bits, bits ^ full, rv, rv ^ full}


def orbit_rep(bits: int, k: int) -> int:
    """The orbit's representative: its lexicographically smallest member, i.e. the
    smallest as an integer (x_0 most significant)."""
    return min(orbit(bits, k))


def r_orbits(n: int, lp: np.ndarray) -> np.ndarray:
    """Algorithm 7 (Appendix A) in the units of r(y) = sum_x p(x) emb(y,x): for every
    input x that represents its orbit and every subsequence y of x,
    r(rep y) += (|O_x| / |O_y|) p(x) emb(y,x); the other outputs of each orbit take
    their representative's value.  Equals the full sum when p is invariant under
    complement and reversal (Theorem 4); dense counts, small n only."""
    E = emb_dense(n)
    p = np.exp(normalise_logp(np.asarray(lp, dtype=float)))
    Y = (1 << (n + 1)) - 1
    r = np.zeros(Y)
    for x in range(1 << n):
        if orbit_rep(x, n) != x:
            continue
        ox = len(orbit(x, n))
        for R in np.nonzero(E[x])[0]:
            yb, k = unrank(int(R))
            oy = len(orbit(yb, k))
            r[rank(orbit_rep(yb, k), k)] += ox / oy * p[x] * E[x, R]
    for R in range(Y):
        yb, k = unrank(R)
        r[R] = r[rank(orbit_rep(yb, k), k)]
    return r


# ---------------------------------------------------------------------------
# Closed forms of the output law for special inputs.
# ---------------------------------------------------------------------------

def r_uniform(n: int) -> np.ndarray:
    """r(y) = sum_x 2^-n emb(y,x) = C(n,k) 2^-k for every y of length k: each of the
    C(n,k) position sets fixes k bits and leaves 2^(n-k) strings."""
    k = output_lengths(n)
    return np.array([math.comb(n, int(kk)) * 2.0 ** (-int(kk)) for kk in k])


def r_product(n: int, pi1: np.ndarray, y_bits: int, k: int) -> float:
    """r(y) = sum_x p(x) emb(y,x) for a product law p(x) = prod_i P(x_i):
    r(y) = sum over position sets S of prod_j P(x_{s_j} = y_j).  Evaluated by the
    recursion over positions f_i(t) = f_{i-1}(t) + f_{i-1}(t-1) P(x_{i-1} = y_{t-1})."""
    y = [(y_bits >> (k - 1 - j)) & 1 for j in range(k)]
    f = [1.0] + [0.0] * k
    for i in range(n):
        for t in range(k, 0, -1):
            pb = pi1[i] if y[t - 1] == 1 else 1.0 - pi1[i]
            f[t] += f[t - 1] * pb
    return f[k]
