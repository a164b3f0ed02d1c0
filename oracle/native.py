"""ctypes loader for the plain-C oracle ``oracle/c/bdc_oracle.c`` (test
infrastructure only; see ``oracle/__init__``).

``build()`` compiles it with gcc and OpenMP into ``oracle/c/libbdc_oracle.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "bdc_oracle.c")
LIB = os.path.join(HERE, "c", "libbdc_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc -O2 -fopenmp).  Returns the library path."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.bdc_row_brute.argtypes = [ctypes.c_int, ctypes.c_uint32, u32p, u32p, ctypes.c_int]
        L.bdc_rows_brute.argtypes = [ctypes.c_int, u32p, ctypes.c_int, u32p, u32p, ctypes.c_int, i32p]
        L.bdc_csr_rowcounts.argtypes = [ctypes.c_int, i64p]
        L.bdc_csr_fill.argtypes = [ctypes.c_int, i64p, u32p, u32p]
        L.bdc_csr_eval.argtypes = [ctypes.c_int, ctypes.c_double, i64p, u32p, u32p, f64p,
                                   ctypes.c_double, ctypes.c_void_p, f64p, f64p]
        L.bdc_csr_iterate.argtypes = [ctypes.c_int, ctypes.c_double, i64p, u32p, u32p, f64p, ctypes.c_int]
        L.bdc_product_r.argtypes = [ctypes.c_int, f64p, ctypes.c_uint32, ctypes.c_int]
        L.bdc_product_r.restype = ctypes.c_double
        L.bdc_product_r_many.argtypes = [ctypes.c_int, f64p, u32p, ctypes.c_int, f64p]
        L.bdc_product_D.argtypes = [ctypes.c_int, ctypes.c_double, f64p, u32p, ctypes.c_int,
                                    f64p, ctypes.c_void_p]
        L.bdc_num_threads.restype = ctypes.c_int
        L.bdc_sample_sweeps.argtypes = [ctypes.c_int, ctypes.c_double, f64p, u32p, ctypes.c_int, f64p,
                                        f64p, f64p]
        L.bdc_sample_sweeps.restype = ctypes.c_longlong
        L.bdc_row_dp.argtypes = [ctypes.c_int, ctypes.c_uint32, u32p, u32p, ctypes.c_int]
        L.bdc_rows_dp.argtypes = [ctypes.c_int, u32p, ctypes.c_int, u32p, u32p, ctypes.c_int, i32p]
        L.bdc_certify.argtypes = [ctypes.c_int, ctypes.c_int, f64p, f64p, ctypes.c_double, f64p, f64p,
                                  ctypes.c_void_p, i64p]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().bdc_num_threads())


def row(n: int, x: int) -> tuple[np.ndarray, np.ndarray]:
    """(ranks, emb) of row x, sorted by rank, by brute force over position subsets."""
    cap = (1 << (n + 1)) - 1
    rk = np.zeros(cap, np.uint32)
    em = np.zeros(cap, np.uint32)
    nnz = lib().bdc_row_brute(n, x, rk, em, cap)
    if nnz < 0:
        raise RuntimeError("bdc_row_brute failed: %d" % nnz)
    return rk[:nnz].copy(), em[:nnz].copy()


def rows(n: int, xs, cap: int | None = None):
    """Several rows at once (OpenMP).  Returns a list of (ranks, emb)."""
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.uint32))
    if cap is None:
        cap = min((1 << (n + 1)) - 1, 40000)
    rk = np.zeros(len(xs) * cap, np.uint32)
    em = np.zeros(len(xs) * cap, np.uint32)
    nnz = np.zeros(len(xs), np.int32)
    rc = lib().bdc_rows_brute(n, xs, len(xs), rk, em, cap, nnz)
    if rc:
        raise RuntimeError("bdc_rows_brute failed: %d" % rc)
    out = []
    for i in range(len(xs)):
        if nnz[i] < 0:
            raise RuntimeError("row capacity %d too small" % cap)
        out.append((rk[i * cap:i * cap + nnz[i]].copy(), em[i * cap:i * cap + nnz[i]].copy()))
    return out


class CSR:
    """The channel's nonzero pattern and embedding counts for n <= 16."""

    def __init__(self, n: int):
        self.n = n
        X = 1 << n
        self.indptr = np.zeros(X + 1, np.int64)
        rc = lib().bdc_csr_rowcounts(n, self.indptr)
        if rc:
            raise RuntimeError("bdc_csr_rowcounts failed: %d" % rc)
        nnz = int(self.indptr[-1])
        self.indices = np.zeros(nnz, np.uint32)
        self.emb = np.zeros(nnz, np.uint32)
        rc = lib().bdc_csr_fill(n, self.indptr, self.indices, self.emb)
        if rc:
            raise RuntimeError("bdc_csr_fill failed: %d" % rc)

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def evaluate(self, d: float, lp: np.ndarray, floor_nats: float = 0.0, want_q: bool = False):
        """(D, L, U, I, q_scaled) in nats at X = exp(lp); see bdc_csr_eval."""
        n = self.n
        lp = np.ascontiguousarray(lp, dtype=np.float64)
        D = np.zeros(1 << n)
        lui = np.zeros(3)
        q = np.zeros((1 << (n + 1)) - 1) if want_q else None
        rc = lib().bdc_csr_eval(n, d, self.indptr, self.indices, self.emb, lp, floor_nats,
                                q.ctypes.data if want_q else None, D, lui)
        if rc:
            raise RuntimeError("bdc_csr_eval failed: %d" % rc)
        return D, float(lui[0]), float(lui[1]), float(lui[2]), q

    def iterate(self, d: float, lp: np.ndarray, iters: int) -> np.ndarray:
        lp = np.array(lp, dtype=np.float64, copy=True)
        rc = lib().bdc_csr_iterate(self.n, d, self.indptr, self.indices, self.emb, lp, iters)
        if rc:
            raise RuntimeError("bdc_csr_iterate failed: %d" % rc)
        return lp


def product_r(n: int, pi1: np.ndarray, ranks) -> np.ndarray:
    ranks = np.ascontiguousarray(np.asarray(ranks, dtype=np.uint32))
    out = np.zeros(len(ranks))
    lib().bdc_product_r_many(n, np.ascontiguousarray(pi1, dtype=np.float64), ranks, len(ranks), out)
    return out


def product_D(n: int, d: float, pi1: np.ndarray, xs, want_Dd: bool = False):
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.uint32))
    D = np.zeros(len(xs))
    Dd = np.zeros(len(xs)) if want_Dd else None
    rc = lib().bdc_product_D(n, d, np.ascontiguousarray(pi1, dtype=np.float64), xs, len(xs), D,
                             Dd.ctypes.data if want_Dd else None)
    if rc:
        raise RuntimeError("bdc_product_D failed: %d" % rc)
    return (D, Dd) if want_Dd else D


def sample_sweeps(n: int, d: float, p: np.ndarray, xs, q_full: np.ndarray):
    """Both sweeps of one BA iteration on the sampled rows xs (brute-force rows).
    Returns (q_part summed over threads, D at xs, nonzeros visited)."""
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.uint32))
    Y = (1 << (n + 1)) - 1
    nt = num_threads()
    q_part = np.zeros(nt * Y)
    D = np.zeros(len(xs))
    tot = lib().bdc_sample_sweeps(n, d, np.ascontiguousarray(p, dtype=np.float64), xs, len(xs),
                                  np.ascontiguousarray(q_full, dtype=np.float64), q_part, D)
    if tot < 0:
        raise RuntimeError("bdc_sample_sweeps failed: %d" % tot)
    return q_part.reshape(nt, Y).sum(axis=0), D, int(tot)


def row_dp(n: int, x: int) -> tuple[np.ndarray, np.ndarray]:
    """(ranks, emb) of row x, sorted by rank, from the per-row subsequence generator
    (NextPos walk with the prefix recurrence of embedding counts)."""
    cap = (1 << (n + 1)) - 1
    rk = np.zeros(cap, np.uint32)
    em = np.zeros(cap, np.uint32)
    nnz = lib().bdc_row_dp(n, x, rk, em, cap)
    if nnz < 0:
        raise RuntimeError("bdc_row_dp failed: %d" % nnz)
    return rk[:nnz].copy(), em[:nnz].copy()


def rows_dp(n: int, xs, cap: int | None = None):
    """Several rows from the generator at once (OpenMP).  Returns a list of (ranks, emb)."""
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.uint32))
    if cap is None:
        cap = min((1 << (n + 1)) - 1, 40000)
    rk = np.zeros(len(xs) * cap, np.uint32)
    em = np.zeros(len(xs) * cap, np.uint32)
    nnz = np.zeros(len(xs), np.int32)
    rc = lib().bdc_rows_dp(n, xs, len(xs), rk, em, cap, nnz)
    if rc:
        raise RuntimeError("bdc_rows_dp failed: %d" % rc)
    out = []
    for i in range(len(xs)):
        if nnz[i] < 0:
            raise RuntimeError("row capacity %d too small" % cap)
        out.append((rk[i * cap:i * cap + nnz[i]].copy(), em[i * cap:i * cap + nnz[i]].copy()))
    return out


def certify(n: int, weights, logps, floor_nats: float = 700.0, want_r: bool = False):
    """Certify-only tier: one FP64 evaluation of Section 2.3 steps 1-2(a) at every
    given law, over every row of the length-n channel (any n <= 22).

    weights: sequence of per-instance length weights w_k (k = 0..n);
    logps: sequence of per-instance log-probabilities (2^n each, any normalisation).
    Returns a dict with L, U, I, M (nats, one per instance), D (count x 2^n, nats),
    r (count x (2^(n+1)-1), if want_r: sum_x e^{lp(x)-M} emb(y,x) of the floored,
    normalised law) and the count statistics of the rows visited."""
    W = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1, n + 1))
    count = W.shape[0]
    LP = np.ascontiguousarray(np.asarray(logps, dtype=np.float64).reshape(count, 1 << n))
    D = np.zeros((count, 1 << n))
    lui = np.zeros((count, 4))
    r = np.zeros((count, (1 << (n + 1)) - 1)) if want_r else None
    stats = np.zeros(5, np.int64)
    rc = lib().bdc_certify(n, count, W, LP, floor_nats, D, lui, r.ctypes.data if want_r else None, stats)
    if rc:
        raise RuntimeError("bdc_certify failed: %d" % rc)
    return {"L": lui[:, 0].copy(), "U": lui[:, 1].copy(), "I": lui[:, 2].copy(), "M": lui[:, 3].copy(),
            "D": D, "r": r,
            "stats": {"nnz": int(stats[0]), "bad_rows": int(stats[1]), "min_row_nnz": int(stats[2]),
                      "max_row_nnz": int(stats[3]), "max_emb": int(stats[4])}}
