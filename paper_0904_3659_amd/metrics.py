"""Throughput conventions for the all-pairs sum.

The paper prices one pair interaction at 38 floating-point operations
(Sec. V-B, discussion of Fig. p) and counts N^2 interactions per force
evaluation.  This package counts the N(N-1) pairs the sum actually has
(j != i) and, for independent systems, the sum of N_s(N_s-1).

Two pair counts matter for a kernel's position against its roofline:
  - ordered pairs (i, j), j != i: the terms of the sum, N(N-1).  A rate in
    ordered pairs per second is the rate at which results are delivered,
    whatever the kernel does to get them;
  - evaluated interactions: what the kernel computes.  A row-gather kernel
    evaluates every ordered pair; a pair-once kernel evaluates each
    unordered pair once and gives the result to both particles, N(N-1)/2.
The fraction of the FP32 peak is quoted on evaluated interactions (38 flop
each for the forward), so that it can never exceed what the arithmetic
units did.
"""

from __future__ import annotations

import numpy as np

FLOP_PER_PAIR = 38
# The adjoint's own count with the same convention: 49 arithmetic flops
# (a fused multiply-add counting 2) plus 19 for the reciprocal square root.
ADJOINT_FLOP_PER_PAIR = 68

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


def is_pair_once(variant: str) -> bool:
    """Whether a kernel variant evaluates each unordered pair once."""
    return variant.startswith(("fwd_sym", "bwd_sym", "bat_sym"))


def evaluated_pairs(ordered_pairs: int, variant: str) -> int:
    """Interactions a variant evaluates to deliver ``ordered_pairs`` terms."""
    return ordered_pairs // 2 if is_pair_once(variant) else ordered_pairs


def gflops(pair_count: float, seconds: float, flop_per_pair: float = FLOP_PER_PAIR) -> float:
    return pair_count * flop_per_pair / seconds / 1e9


def frac_of_fp32_peak(pairs_per_second: float, flop_per_pair: float = FLOP_PER_PAIR) -> float:
    return pairs_per_second * flop_per_pair / (MI355X_FP32_VECTOR_TFLOPS * 1e12)
