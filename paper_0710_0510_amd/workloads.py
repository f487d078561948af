"""Seeded synthetic inputs for the Q-adic transform path.

This module holds workload descriptions and random-number draws only: no
packing, no reduction, no field arithmetic.  Both the HIP library's callers
and the CPU oracle take their inputs from here.

Element format: uint8 coefficients, k bytes per element (byte i is the
coefficient of X^i), every value uniform in [0, p); matrices row-major.
Draws use numpy's PCG64 (``numpy.random.default_rng(seed)``).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np


@dataclass(frozen=True)
class Field:
    p: int
    k: int
    P_low: Tuple[int, ...]   # low coefficients of the monic defining polynomial

    @property
    def name(self) -> str:
        return f"GF({self.p}^{self.k})"


# Defining polynomials (low coefficients first, monic leading term implied).
GF7_2 = Field(7, 2, (1, 0))          # X^2 + 1
GF3_4 = Field(3, 4, (2, 0, 0, 2))    # X^4 + 2X^3 + 2
GF5_3 = Field(5, 3, (3, 3, 0))       # X^3 + 3X + 3
GF3_2 = Field(3, 2, (1, 0))          # X^2 + 1


@dataclass(frozen=True)
class Workload:
    name: str
    kind: str                 # "polymul" | "gemm" | "batched" | "dfqt" | "dfqt_batched" | "transforms"
    p: int
    k: int
    P_low: Tuple[int, ...] = ()
    seed: int = 0
    n: int = 0                # polymul: number of products
    q: int = 0                # polymul: radix given by the workload
    M: int = 0
    N: int = 0
    K: int = 0
    count: int = 0            # batched: number of products
    lo: int = 0               # batched: M, N, K uniform in [lo, hi]
    hi: int = 0
    length: int = 0           # dfqt: coefficients per operand (degree N = length - 1)
    d: int = 0                # dfqt: chunks of d + 1 coefficients
                              # dfqt_batched: lengths uniform in [lo, hi], count pairs


WORKLOADS = {
    "polymul-gf5-k3": Workload("polymul-gf5-k3", "polymul", 5, 3, (), seed=1, n=65536, q=64),
    # the same products scaled to 2^24 pairs: large enough to stream at HBM rate
    "polymul-gf5-k3-2^24": Workload("polymul-gf5-k3-2^24", "polymul", 5, 3, (), seed=1,
                                    n=1 << 24, q=64),
    "gemm-gf7^2-1024": Workload("gemm-gf7^2-1024", "gemm", 7, 2, GF7_2.P_low, seed=2,
                                M=1024, N=1024, K=1024),
    "batched-gf3^4-4096": Workload("batched-gf3^4-4096", "batched", 3, 4, GF3_4.P_low,
                                   seed=3, count=4096, lo=16, hi=256),
    "gemm-gf5^3-4096": Workload("gemm-gf5^3-4096", "gemm", 5, 3, GF5_3.P_low, seed=4,
                                M=4096, N=4096, K=4096),
    "gemm-gf3^2-8192": Workload("gemm-gf3^2-8192", "gemm", 3, 2, GF3_2.P_low, seed=5,
                                M=8192, N=8192, K=8192),
    # long polynomials over GF(3): degree N = 500, d = 4 (the paper's Fig. 2 case),
    # a batch of independent pairs
    "dfqt-gf3-n500-d4": Workload("dfqt-gf3-n500-d4", "dfqt", 3, 1, (), seed=6, count=16384,
                                 length=501, d=4),
    # uneven pairs over GF(3): both operand lengths drawn independently,
    # uniform in 1..1024 coefficients, one persistent launch for the batch
    "dfqt-uneven-gf3-1024": Workload("dfqt-uneven-gf3-1024", "dfqt_batched", 3, 1, (), seed=8,
                                     count=16384, lo=1, hi=1024, d=4),
    # the boundary's standalone transforms on 2^24 elements of GF(5^3) at
    # q = 2^6: DQT pack of coefficient bytes, REDQ unpack of values with
    # 2k - 1 = 5 base-q digits to polynomial digits and to field elements
    "transforms-gf5^3-2^24": Workload("transforms-gf5^3-2^24", "transforms", 5, 3, GF5_3.P_low,
                                      seed=9, n=1 << 24, q=64),
}


def coeffs(rng: np.random.Generator, shape, p: int, k: int) -> np.ndarray:
    """uint8 array of shape (*shape, k), i.i.d. uniform in [0, p)."""
    return rng.integers(0, p, size=tuple(shape) + (k,), dtype=np.uint8)


def polymul_inputs(w: Workload):
    rng = np.random.default_rng(w.seed)
    a = coeffs(rng, (w.n,), w.p, w.k)
    b = coeffs(rng, (w.n,), w.p, w.k)
    return a, b


def transform_inputs(w: Workload):
    """n elements' coefficient bytes (uniform in [0, p)) for the pack, and n
    integers uniform in [0, q^(2k-1)) as binary64 (exact: q^(2k-1) <= 2^53)
    for the unpack."""
    rng = np.random.default_rng(w.seed)
    c = coeffs(rng, (w.n,), w.p, w.k)
    top = w.q ** (2 * w.k - 1)
    assert top <= 1 << 53
    r = rng.integers(0, top, size=w.n, dtype=np.int64).astype(np.float64)
    return c, r


def poly_long_inputs(w: Workload, count: int = 0):
    """count x length coefficient arrays a, b, i.i.d. uniform in [0, p)."""
    count = count or w.count
    rng = np.random.default_rng(w.seed)
    a = rng.integers(0, w.p, size=(count, w.length), dtype=np.uint8)
    b = rng.integers(0, w.p, size=(count, w.length), dtype=np.uint8)
    return a, b


def poly_uneven_lengths(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    """count x 2 int64 array of operand lengths (la, lb), each uniform in
    [lo, hi], drawn before any coefficient."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(count, 2)).astype(np.int64)


def poly_uneven_inputs(w: Workload, count: int = 0):
    """Lengths first (as poly_uneven_lengths), then every first operand as
    one flat array (pair i at offset sum of the earlier la), then every
    second operand likewise; coefficients i.i.d. uniform in [0, p)."""
    count = count or w.count
    rng = np.random.default_rng(w.seed)
    lens = rng.integers(w.lo, w.hi + 1, size=(count, 2)).astype(np.int64)
    a = rng.integers(0, w.p, size=int(lens[:, 0].sum()), dtype=np.uint8)
    b = rng.integers(0, w.p, size=int(lens[:, 1].sum()), dtype=np.uint8)
    return lens, a, b


def gemm_inputs(w: Workload, M: int = 0, N: int = 0, K: int = 0):
    """A (M x K x k) and B (K x N x k); smaller shapes draw a prefix-free
    stream of their own (same seed, fewer draws)."""
    M, N, K = M or w.M, N or w.N, K or w.K
    rng = np.random.default_rng(w.seed)
    A = coeffs(rng, (M, K), w.p, w.k)
    B = coeffs(rng, (K, N), w.p, w.k)
    return A, B


def batched_shapes(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    """count x 3 array of (M, N, K), each uniform in [lo, hi], drawn before
    any entry."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(count, 3))


def batched_inputs(w: Workload, count: int = 0):
    """Shapes first, then per product in order A (M x K x k), B (K x N x k)
    from the same generator."""
    count = count or w.count
    rng = np.random.default_rng(w.seed)
    mnk = rng.integers(w.lo, w.hi + 1, size=(count, 3))
    As: List[np.ndarray] = []
    Bs: List[np.ndarray] = []
    for (M, N, K) in mnk.tolist():
        As.append(coeffs(rng, (M, K), w.p, w.k))
        Bs.append(coeffs(rng, (K, N), w.p, w.k))
    return mnk, As, Bs


def random_matrix(seed: int, shape, p: int, k: int) -> np.ndarray:
    return coeffs(np.random.default_rng(seed), shape, p, k)
