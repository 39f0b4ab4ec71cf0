"""Throughput conventions for the all-pairs sum.

The paper prices one pair interaction at 38 floating-point operations
(Sec. V-B, discussion of Fig. p) and counts N^2 interactions per force
evaluation.  This package counts the N(N-1) pairs the sum actually has
(j != i) and, for independent systems, the sum of N_s(N_s-1).
"""

from __future__ import annotations

import numpy as np

FLOP_PER_PAIR = 38

# MI355X published peaks (dense, no sparsity).
MI355X_FP32_VECTOR_TFLOPS = 157.3
MI355X_HBM_TBPS = 8.0


def pairs(n: int) -> int:
    """Ordered pairs (i, j), j != i, of one system of n particles."""
    n = int(n)
    return n * (n - 1) if n > 1 else 0


def pairs_ensemble(sizes) -> int:
    s = np.asarray(sizes, dtype=np.int64)
    return int(np.sum(s * np.maximum(s - 1, 0)))


def gflops(pair_count: float, seconds: float, flop_per_pair: float = FLOP_PER_PAIR) -> float:
    return pair_count * flop_per_pair / seconds / 1e9


def frac_of_fp32_peak(pairs_per_second: float, flop_per_pair: float = FLOP_PER_PAIR) -> float:
    return pairs_per_second * flop_per_pair / (MI355X_FP32_VECTOR_TFLOPS * 1e12)
