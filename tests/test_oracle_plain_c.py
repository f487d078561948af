"""The multi-core C schoolbook comparator (oracle/plain_gf.c) against the
Python oracle: the same field products by an independent implementation."""
import numpy as np
import pytest

from oracle import gf, plain_c

FIELDS = [(7, 2, (1, 0)), (3, 4, (2, 0, 0, 2)), (5, 3, (3, 3, 0)), (13, 1, (11,)),
          (2, 4, (1, 0, 0, 1)), (13, 3, (1, 0, 4)), (61, 2, (59, 0))]


@pytest.mark.parametrize("p,k,P", FIELDS)
def test_gemm_matches_one_product_at_a_time(p, k, P):
    assert gf.is_irreducible(P, p)
    rng = np.random.default_rng(p * 10 + k)
    A = rng.integers(0, p, size=(5, 7, k), dtype=np.uint8)
    B = rng.integers(0, p, size=(7, 4, k), dtype=np.uint8)
    want = np.array(gf.gemm_gfpk_small(A.tolist(), B.tolist(), p, P), dtype=np.uint8)
    assert np.array_equal(plain_c.gemm(A, B, p, P, threads=3), want)


@pytest.mark.parametrize("p,k,P", FIELDS)
def test_gemm_matches_planes_all_extremes(p, k, P):
    rng = np.random.default_rng(k)
    A = rng.integers(0, p, size=(33, 70, k), dtype=np.uint8)
    B = rng.integers(0, p, size=(70, 19, k), dtype=np.uint8)
    A[0] = p - 1
    B[:, 0] = p - 1
    assert np.array_equal(plain_c.gemm(A, B, p, P), gf.gemm_gfpk_planes(A, B, p, P))


def test_gemm_identity_and_empty():
    p, k, P = 5, 3, (3, 3, 0)
    rng = np.random.default_rng(3)
    A = rng.integers(0, p, size=(9, 6, k), dtype=np.uint8)
    eye = np.zeros((6, 6, k), dtype=np.uint8)
    eye[np.arange(6), np.arange(6), 0] = 1
    assert np.array_equal(plain_c.gemm(A, eye, p, P), A)
    assert plain_c.gemm(A[:, :0], eye[:0], p, P).sum() == 0  # K = 0: zero matrix
    assert plain_c.gemm(A[:0], eye, p, P).shape == (0, 6, k)


def test_batched_matches_products():
    p, k, P = 3, 4, (2, 0, 0, 2)
    rng = np.random.default_rng(11)
    shapes = [(3, 5, 2), (17, 1, 9), (1, 1, 1), (8, 12, 0), (20, 13, 31)]
    As = [rng.integers(0, p, size=(M, K, k), dtype=np.uint8) for M, N, K in shapes]
    Bs = [rng.integers(0, p, size=(K, N, k), dtype=np.uint8) for M, N, K in shapes]
    outs = plain_c.gemm_batched(As, Bs, p, P, threads=2)
    for a, b, c in zip(As, Bs, outs):
        assert np.array_equal(c, gf.gemm_gfpk_planes(a, b, p, P))


def test_polymul_matches_oracle_and_exhaustive_gf5_k2():
    rng = np.random.default_rng(5)
    a = rng.integers(0, 5, size=(1000, 3), dtype=np.uint8)
    b = rng.integers(0, 5, size=(1000, 3), dtype=np.uint8)
    assert np.array_equal(plain_c.polymul_batch(a, b, 5), gf.polymul_batch(a, b, 5))
    pairs = np.array([(x, y, u, v) for x in range(5) for y in range(5)
                      for u in range(5) for v in range(5)], dtype=np.uint8)
    c = plain_c.polymul_batch(pairs[:, :2], pairs[:, 2:], 5)
    for (x, y, u, v), row in zip(pairs.tolist(), c.tolist()):
        assert row == [x * u % 5, (x * v + y * u) % 5, y * v % 5]


def test_threads_reported_and_bad_arguments():
    A = np.zeros((4, 3, 2), dtype=np.uint8)
    B = np.zeros((3, 2, 2), dtype=np.uint8)
    plain_c.gemm(A, B, 7, (1, 0), threads=2)
    assert plain_c.threads_used() == 2
    with pytest.raises(ValueError):
        plain_c.gemm(A, B, 1, (1, 0))   # p < 2
    with pytest.raises(ValueError):
        plain_c.polymul_batch(np.zeros((2, 9), np.uint8), np.zeros((2, 9), np.uint8), 3)  # k > 8
