"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no arithmetic of the Blahut-Arimoto method itself: it only
draws seeded random numbers and lays them out.  Both the CPU oracle tests and
the GPU path receive the same arrays from here, so that parity compares the two
implementations on identical inputs.

String convention (used everywhere in this repository): an input string
x = (x_0, ..., x_{n-1}) is stored as the integer sum_i x_i * 2^(n-1-i), so x_0 is
the most significant bit and lexicographic order equals numeric order.
"""
from __future__ import annotations

import numpy as np

N_MAX = 20


def d_grid(lo: float = 0.64, hi: float = 0.96, count: int = 32) -> np.ndarray:
    """Deletion probabilities evenly spaced in [lo, hi], endpoints included."""
    return np.linspace(lo, hi, count)


def theta_normal(n: int, seed: int = 0, sigma: float = 0.1) -> np.ndarray:
    """Logits theta ~ N(0, sigma^2) for the 2^n inputs, float64, from numpy's PCG64."""
    return np.random.default_rng(seed).normal(0.0, sigma, 1 << n)


def sample_rows(n: int, count: int, seed: int = 1) -> np.ndarray:
    """Seeded input strings for sampled-row checks.

    Always contains the structured extremes (all zeros, all ones, the two
    alternating strings, a single run boundary) followed by uniform draws."""
    full = (1 << n) - 1
    alt = 0
    for i in range(n):
        alt = (alt << 1) | (i & 1)
    fixed = [0, full, alt, full ^ alt, (1 << (n // 2)) - 1 if n > 1 else 0]
    rng = np.random.default_rng(seed)
    rest = rng.integers(0, 1 << n, size=max(count - len(fixed), 0), dtype=np.int64)
    out = np.unique(np.concatenate([np.array(fixed, dtype=np.int64), rest]))
    return out[:count] if len(out) > count else out


def sample_outputs(n: int, count: int, seed: int = 2) -> np.ndarray:
    """Seeded output ranks in [0, 2^(n+1)-1) for sampled-output checks (includes
    the empty string, rank 0, and the last rank)."""
    rng = np.random.default_rng(seed)
    top = (1 << (n + 1)) - 1
    rest = rng.integers(0, top, size=max(count - 2, 0), dtype=np.int64)
    return np.unique(np.concatenate([np.array([0, top - 1], dtype=np.int64), rest]))


def product_bit_probs(n: int, seed: int = 3, lo: float = 0.15, hi: float = 0.85) -> np.ndarray:
    """Per-position probabilities P(x_i = 1), drawn uniformly in [lo, hi]."""
    return np.random.default_rng(seed).uniform(lo, hi, n)


def product_logp(n: int, pi1: np.ndarray) -> np.ndarray:
    """log of the product distribution p(x) = prod_i P(x_i), float64, length 2^n.

    Layout only: x_i is bit (n-1-i) of the index."""
    x = np.arange(1 << n, dtype=np.int64)
    lp = np.zeros(1 << n)
    for i in range(n):
        bit = (x >> (n - 1 - i)) & 1
        lp += np.where(bit == 1, np.log(pi1[i]), np.log1p(-pi1[i]))
    return lp


def random_logp(n: int, seed: int = 4, spread: float = 3.0) -> np.ndarray:
    """Unnormalised log-probabilities with a wide dynamic range (normal, std `spread`)."""
    return np.random.default_rng(seed).normal(0.0, spread, 1 << n)
