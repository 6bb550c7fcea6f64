"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle leg.

This module draws random numbers and nothing else: it holds none of the
method's arithmetic (no words, arcs, (min,+) products or traces), so both the
CPU oracle and the HIP path can be fed from it without sharing code.

Workloads (every one is synthetic; the paper's own inputs are generated from
the path order n alone):

* ``raw_gemm_pair``   -- two square uint16 matrices for the raw (min,+) product
  benchmark: entries uniform in 0..24, 30 % of them set to INF = 65535,
  ``numpy.random.default_rng(seed)``, A drawn before B.
* ``stress_matrix``   -- matrices for parity stress tests (wide value ranges,
  chosen INF fractions, sums near INF).
* ``residual_matrix`` -- 8-bit residuals with one shared base (and optionally
  one offset per row) for the compact-power steps: uniform residuals in
  [lo, hi] with the least value placed at least once.
* ``batch_instances`` -- the mixed batch: 64 (n, m) pairs, n uniform in 4..9,
  m uniform in 3..200, n drawn before m.
* ``serve_stream``    -- a Poisson stream of (arrival time, n, m) queries with
  n in 6..12 weighted by 2^-(n-6) and m uniform in 3..500.
"""
from __future__ import annotations

import numpy as np

INF16 = 65535
INF8 = 255


def raw_gemm_pair(N: int, seed: int = 0, hi: int = 24, inf_frac: float = 0.3):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(2):
        X = rng.integers(0, hi + 1, size=(N, N), dtype=np.uint16)
        X[rng.random((N, N)) < inf_frac] = INF16
        out.append(X)
    return out[0], out[1]


def stress_matrix(rows: int, cols: int, seed: int, lo: int = 0, hi: int = 30000,
                  inf_frac: float = 0.3, dtype=np.uint16) -> np.ndarray:
    """Uniform entries in [lo, hi] with a fraction set to the dtype's INF."""
    inf = INF16 if dtype == np.uint16 else INF8
    hi = min(hi, inf - 1)
    rng = np.random.default_rng(seed)
    X = rng.integers(lo, hi + 1, size=(rows, cols)).astype(dtype)
    if inf_frac > 0:
        X[rng.random((rows, cols)) < inf_frac] = inf
    return X


def residual_matrix(rows: int, cols: int, seed: int, lo: int = 0, hi: int = 14,
                    base: int = 600, row_offsets: tuple | None = None):
    """(x, base_word, offsets): x uint8 rows x cols uniform in [lo, hi] with
    x[0, 0] = lo, so lo is the least residual; base_word = int32 [base, lo];
    offsets = int32 per-row values uniform in row_offsets (inclusive), or
    None when row_offsets is None."""
    rng = np.random.default_rng(seed)
    x = rng.integers(lo, hi + 1, size=(rows, cols)).astype(np.uint8)
    if rows and cols:
        x[0, 0] = lo
    word = np.array([base, lo], dtype=np.int32)
    off = None
    if row_offsets is not None:
        off = rng.integers(row_offsets[0], row_offsets[1] + 1, size=rows).astype(np.int32)
    return x, word, off


def batch_instances(seed: int = 0, count: int = 64, n_lo: int = 4, n_hi: int = 9,
                    m_lo: int = 3, m_hi: int = 200):
    rng = np.random.default_rng(seed)
    n = rng.integers(n_lo, n_hi + 1, size=count)
    m = rng.integers(m_lo, m_hi + 1, size=count)
    return [(int(a), int(b)) for a, b in zip(n, m)]


def serve_stream(seed: int = 0, count: int = 2000, qps: float = 100.0, n_lo: int = 6,
                 n_hi: int = 12, m_lo: int = 3, m_hi: int = 500):
    """List of (arrival_seconds, n, m); inter-arrival times ~ Exp(1/qps)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=count)
    ns = np.arange(n_lo, n_hi + 1)
    w = 2.0 ** (-(ns - n_lo).astype(np.float64))
    n = rng.choice(ns, size=count, p=w / w.sum())
    m = rng.integers(m_lo, m_hi + 1, size=count)
    t = np.cumsum(gaps)
    return [(float(a), int(b), int(c)) for a, b, c in zip(t, n, m)]
